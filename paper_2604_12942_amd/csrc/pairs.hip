// Per-pair screen-space gradients from the render backward's per-instance records: the records of
// one (view, Gaussian) pair are contiguous in emission order, so a pair's gradient is a
// fixed-order sum that needs no atomics.
#include "gsr_internal.h"

namespace gsr {

__global__ void k_zero_f32(float *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = 0.f;
}

// Per-pair screen-space gradient: the fixed-order sum of the pair's instance records.
// Small pairs (at most kSmallPair records): each wave takes 64 consecutive visible pairs in
// emission order.  Their records form one contiguous run, which the wave streams through LDS
// kWinRecs records at a time with coalesced loads (a window that holds no record of a small pair
// is not loaded), and each lane adds its own pair's records from there, in order.
// Large pairs (near Gaussians cover hundreds of tiles, and depth order puts them first): each is
// summed by one whole wave, each lane striding over the records and a lane tree adding the 64
// partial sums.  The large pairs are dealt out across the grid: lane l of wave w looks at pair
// w + l W (W waves in the grid), so the large pairs at the front of the list go to different waves
// rather than queueing in the first ones.  Either way the order of the additions is fixed by the
// data, so the result repeats exactly.
constexpr uint32_t kSmallPair = 64;
constexpr int kPairWaves = 4;  // waves per workgroup
constexpr int kWinRecs = 256;  // records per LDS window of a wave

__device__ __forceinline__ uint32_t pair_count(const uint32_t *__restrict__ pair_gid,
                                               const uint32_t *__restrict__ pair_first,
                                               const uint32_t *__restrict__ ntiles, uint32_t q, uint32_t np,
                                               uint32_t first) {
    // a pair's records end where the next pair's begin (the last pair: its tile count)
    return q + 1 < np ? pair_first[q + 1] - first : ntiles[pair_gid[q]];
}

__global__ __launch_bounds__(64 * kPairWaves) void k_pair_grads(const float *__restrict__ dinst,
                                                                const uint32_t *__restrict__ pair_gid,
                                                                const uint32_t *__restrict__ pair_first,
                                                                const uint32_t *__restrict__ n_pairs,
                                                                const uint32_t *__restrict__ ntiles,
                                                                float *__restrict__ dsplat) {
    // one window of records per wave: floats 0-3 and 4-7 of each record as float4, 8-9 as float2
    __shared__ float4 s_w4[kPairWaves][2][kWinRecs];
    __shared__ float2 s_w2[kPairWaves][kWinRecs];
    const uint32_t np = *n_pairs;
    const int lane = __lane_id();
    const uint32_t gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    float4 *const w4a = s_w4[threadIdx.x >> 6][0], *const w4b = s_w4[threadIdx.x >> 6][1];
    float2 *const w2 = s_w2[threadIdx.x >> 6];
    // small pairs, one per lane
    for (uint32_t w0 = gw * 64; w0 < np; w0 += nwaves * 64) {
        const uint32_t q = w0 + lane;
        const bool live = q < np;
        const uint32_t first = live ? pair_first[q] : 0u;
        const uint32_t cnt = live ? pair_count(pair_gid, pair_first, ntiles, q, np, first) : 0u;
        const bool small = live && cnt <= kSmallPair;
        // the run of records of the wave's pairs: from the first pair's first record to the end
        // of the last live pair
        const int lastl = np - w0 < 64u ? (int)(np - w0) - 1 : 63;
        const uint32_t r0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)first);
        const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)(first + cnt), lastl);
        float acc[GSR_SPLAT_GRAD_FLOATS];
#pragma unroll
        for (int e = 0; e < GSR_SPLAT_GRAD_FLOATS; e++) acc[e] = 0.f;
        for (uint32_t a = r0; a < r1; a += kWinRecs) {
            // this lane's records inside the window [a, a + kWinRecs)
            const uint32_t k0 = first > a ? first : a;
            const uint32_t k1 = first + cnt < a + kWinRecs ? first + cnt : a + kWinRecs;
            const bool need = small && k0 < k1;
            if (__ballot(need) == 0) continue;
            float2 x[kWinRecs / 64][5];
#pragma unroll
            for (int u = 0; u < kWinRecs / 64; u++)
                if (a + u * 64 + lane < r1) {
                    const float2 *rec = reinterpret_cast<const float2 *>(
                        dinst + (int64_t)(a + u * 64 + lane) * GSR_SPLAT_GRAD_FLOATS);
#pragma unroll
                    for (int e = 0; e < 5; e++) x[u][e] = rec[e];
                }
#pragma unroll
            for (int u = 0; u < kWinRecs / 64; u++)
                if (a + u * 64 + lane < r1) {
                    const int s = u * 64 + lane;
                    w4a[s] = make_float4(x[u][0].x, x[u][0].y, x[u][1].x, x[u][1].y);
                    w4b[s] = make_float4(x[u][2].x, x[u][2].y, x[u][3].x, x[u][3].y);
                    w2[s] = x[u][4];
                }
            __builtin_amdgcn_wave_barrier();  // the wave reads back what its lanes just wrote
            if (need)
                for (uint32_t k = k0; k < k1; k++) {
                    const int s = (int)(k - a);
                    const float4 xa = w4a[s], xb = w4b[s];
                    const float2 xc = w2[s];
                    acc[0] += xa.x;
                    acc[1] += xa.y;
                    acc[2] += xa.z;
                    acc[3] += xa.w;
                    acc[4] += xb.x;
                    acc[5] += xb.y;
                    acc[6] += xb.z;
                    acc[7] += xb.w;
                    acc[8] += xc.x;
                    acc[9] += xc.y;
                }
            __builtin_amdgcn_wave_barrier();  // every read of the window precedes the next window's writes
        }
        if (small) {
            float2 *out = reinterpret_cast<float2 *>(dsplat + (int64_t)pair_gid[q] * GSR_SPLAT_GRAD_FLOATS);
#pragma unroll
            for (int e = 0; e < 5; e++) out[e] = make_float2(acc[2 * e], acc[2 * e + 1]);
        }
    }
    // large pairs, one per wave, dealt out across the grid
    for (uint32_t k0 = 0; (uint64_t)k0 * nwaves + gw < np; k0 += 64) {
        const uint64_t qq = (uint64_t)(k0 + lane) * nwaves + gw;
        const bool live = qq < np;
        const uint32_t q = live ? (uint32_t)qq : 0u;
        const uint32_t first = live ? pair_first[q] : 0u;
        const uint32_t cnt = live ? pair_count(pair_gid, pair_first, ntiles, q, np, first) : 0u;
        uint64_t big = __ballot(live && cnt > kSmallPair);
        while (big) {
            const int src = __builtin_ctzll(big);
            big &= big - 1;
            const uint32_t bq = (uint32_t)__builtin_amdgcn_readlane((int)q, src);
            const uint32_t bf = (uint32_t)__builtin_amdgcn_readlane((int)first, src);
            const uint32_t bc = (uint32_t)__builtin_amdgcn_readlane((int)cnt, src);
            const uint32_t bg = pair_gid[bq];
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
    const int nb = (int)(ceil_div(VN, 64 * kPairWaves) < 8192 ? ceil_div(VN, 64 * kPairWaves) : 8192);
    k_pair_grads<<<nb, 64 * kPairWaves, 0, st>>>(dinst, em->pair_gid, em->pair_first, em->n_pairs, tile_info, dsplat);
    return last_launch();
}

