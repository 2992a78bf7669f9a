// Per-pair screen-space gradients from the render backward's per-instance records: the records of
// one (view, Gaussian) pair are contiguous in emission order, so a pair's gradient is a
// fixed-order sum that needs no atomics.
#include "gsr_internal.h"

namespace gsr {

__global__ void k_zero_f32(float *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = 0.f;
}

// Per-pair screen-space gradient: the fixed-order sum of the pair's instance records.  Each
// wave takes 64 consecutive visible pairs in emission order.  A pair of at most kSmallPair
// records is summed by its own lane, four records in flight; the wave's larger pairs (near
// Gaussians cover hundreds of tiles) are then summed one after the other by the whole wave, each
// lane striding over the records and a lane tree adding the 64 partial sums.  Either way the
// order of the additions is fixed by the data, so the result repeats exactly.
constexpr uint32_t kSmallPair = 32;

__global__ __launch_bounds__(256) void k_pair_grads(const float *__restrict__ dinst,
                                                    const uint32_t *__restrict__ pair_gid,
                                                    const uint32_t *__restrict__ pair_first,
                                                    const uint32_t *__restrict__ n_pairs,
                                                    const uint32_t *__restrict__ ntiles, float *__restrict__ dsplat) {
    const uint32_t np = *n_pairs;
    const int lane = __lane_id();
    const uint32_t wave0 = (blockIdx.x * blockDim.x + threadIdx.x) & ~63u;
    const uint32_t wstride = gridDim.x * blockDim.x;
    for (uint32_t w0 = wave0; w0 < np; w0 += wstride) {
        const uint32_t q = w0 + lane;
        const bool live = q < np;
        const uint32_t gid = live ? pair_gid[q] : 0u;
        const uint32_t first = live ? pair_first[q] : 0u;
        // a pair's records end where the next pair's begin (a coalesced read instead of a gather
        // of the pair's tile count, which only the last pair needs)
        const uint32_t cnt = !live ? 0u : q + 1 < np ? pair_first[q + 1] - first : ntiles[gid];
        const bool small = cnt <= kSmallPair;
        if (live && small) {
            const float2 *rec = reinterpret_cast<const float2 *>(dinst + (int64_t)first * GSR_SPLAT_GRAD_FLOATS);
            float acc[GSR_SPLAT_GRAD_FLOATS];
#pragma unroll
            for (int e = 0; e < GSR_SPLAT_GRAD_FLOATS; e++) acc[e] = 0.f;
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
        // the wave's large pairs, one at a time
        uint64_t big = __ballot(live && !small);
        while (big) {
            const int src = __builtin_ctzll(big);
            big &= big - 1;
            const uint32_t bf = (uint32_t)__builtin_amdgcn_readlane((int)first, src);
            const uint32_t bc = (uint32_t)__builtin_amdgcn_readlane((int)cnt, src);
            const uint32_t bg = (uint32_t)__builtin_amdgcn_readlane((int)gid, src);
            float acc[GSR_SPLAT_GRAD_FLOATS];
#pragma unroll
            for (int e = 0; e < GSR_SPLAT_GRAD_FLOATS; e++) acc[e] = 0.f;
            for (uint32_t j = lane; j < bc; j += 64) {
                const float2 *rec =
                    reinterpret_cast<const float2 *>(dinst + ((int64_t)bf + j) * GSR_SPLAT_GRAD_FLOATS);
#pragma unroll
                for (int e = 0; e < 5; e++) {
                    const float2 x = rec[e];
                    acc[2 * e] += x.x;
                    acc[2 * e + 1] += x.y;
                }
            }
#pragma unroll
            for (int e = 0; e < GSR_SPLAT_GRAD_FLOATS; e++) acc[e] = wave_sum(acc[e]);
            if (lane == 0) {
                float2 *out = reinterpret_cast<float2 *>(dsplat + (int64_t)bg * GSR_SPLAT_GRAD_FLOATS);
#pragma unroll
                for (int e = 0; e < 5; e++) out[e] = make_float2(acc[2 * e], acc[2 * e + 1]);
            }
        }
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
    const int nb = (int)(ceil_div(VN, 256) < 8192 ? ceil_div(VN, 256) : 8192);
    k_pair_grads<<<nb, 256, 0, st>>>(dinst, em->pair_gid, em->pair_first, em->n_pairs, tile_info, dsplat);
    return last_launch();
}

