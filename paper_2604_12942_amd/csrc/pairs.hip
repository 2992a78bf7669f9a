// Per-pair screen-space gradients from the render backward's per-instance records: the records of
// one (view, Gaussian) pair are contiguous in emission order, so a pair's gradient is a
// fixed-order sum that needs no atomics.
#include "gsr_internal.h"

namespace gsr {

__global__ void k_zero_f32(float *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = 0.f;
}

// Per-pair screen-space gradient: the fixed-order sum of the pair's instance records.  One
// thread per visible pair in emission order, so a wave reads one contiguous run of records.
__global__ void k_pair_grads(const float *__restrict__ dinst, const uint32_t *__restrict__ pair_gid,
                             const uint32_t *__restrict__ pair_first, const uint32_t *__restrict__ n_pairs,
                             const uint32_t *__restrict__ ntiles, float *__restrict__ dsplat) {
    const uint32_t np = *n_pairs;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < np; q += gridDim.x * blockDim.x) {
        const uint32_t gid = pair_gid[q];
        const uint32_t cnt = ntiles[gid];
        const float2 *rec = reinterpret_cast<const float2 *>(dinst + (int64_t)pair_first[q] * GSR_SPLAT_GRAD_FLOATS);
        float acc[GSR_SPLAT_GRAD_FLOATS];
#pragma unroll
        for (int e = 0; e < GSR_SPLAT_GRAD_FLOATS; e++) acc[e] = 0.f;
        // four records in flight per step (the additions keep the fixed order)
        uint32_t j = 0;
        for (; j + 4 <= cnt; j += 4) {
            float2 x[4][5];
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int e = 0; e < 5; e++) x[u][e] = rec[(j + u) * 5 + e];
#pragma unroll
            for (int u = 0; u < 4; u++)
#pragma unroll
                for (int e = 0; e < 5; e++) {
                    acc[2 * e] += x[u][e].x;
                    acc[2 * e + 1] += x[u][e].y;
                }
        }
        for (; j < cnt; j++)
#pragma unroll
            for (int e = 0; e < 5; e++) {
                const float2 x = rec[j * 5 + e];
                acc[2 * e] += x.x;
                acc[2 * e + 1] += x.y;
            }
        float2 *out = reinterpret_cast<float2 *>(dsplat + (int64_t)gid * GSR_SPLAT_GRAD_FLOATS);
#pragma unroll
        for (int e = 0; e < 5; e++) out[e] = make_float2(acc[2 * e], acc[2 * e + 1]);
    }
}

}  // namespace gsr

using namespace gsr;

// all_pairs: zero the pairs that were not rendered first (else they are left untouched).
extern "C" gsr_status gsr_pair_grads_launch(const float *dinst, const gsr_emission *em, const uint32_t *tile_info,
                                            int64_t VN, float *dsplat, bool all_pairs, hipStream_t st) {
    if (VN <= 0) return GSR_OK;
    if (all_pairs) {
        const int64_t words = VN * GSR_SPLAT_GRAD_FLOATS;
        const int nz = (int)(ceil_div(words, 256) < 16384 ? ceil_div(words, 256) : 16384);
        k_zero_f32<<<nz, 256, 0, st>>>(dsplat, words);
    }
    const int nb = (int)(ceil_div(VN, 256) < 16384 ? ceil_div(VN, 256) : 16384);
    k_pair_grads<<<nb, 256, 0, st>>>(dinst, em->pair_gid, em->pair_first, em->n_pairs, tile_info, dsplat);
    return last_launch();
}

