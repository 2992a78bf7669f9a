// Internal helpers of libgsr (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsr.h"

#define GSR_LOG2E 1.4426950408889634
#define GSR_LN2 0.6931471805599453
// blend-weight exponent scale: exp(-x/2) = 2^(-x * log2(e) / 2)
#define GSR_KAPPA (0.5 * GSR_LOG2E)
#define GSR_ALPHA_MAX 0.99f
#define GSR_T_MIN 1e-4f
#define GSR_LOWPASS 0.3
#define GSR_GUARD 1.3

namespace gsr {

// Launch bookkeeping: every entry point returns GSR_E_HIP if a launch failed.
inline gsr_status last_launch() { return hipGetLastError() == hipSuccess ? GSR_OK : GSR_E_HIP; }

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline bool valid_tile(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 8 && th == 32) || (tw == 32 && th == 8);
}

// Sort / scan geometry shared by the binning kernels.
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // 4096 keys per block
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// ---- wave64 helpers --------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() {
    return (__lane_id() == 0) ? 0ull : (~0ull >> (64 - __lane_id()));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Inclusive scan across the wave (lane order).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t o = __shfl_up(v, off);
        if (__lane_id() >= (unsigned)off) v += o;
    }
    return v;
}

// Exclusive scan of one value per thread over a 256-thread block.  Returns the exclusive
// prefix; *total (optional) receives the block sum.  Uses 4 words of LDS and two barriers.
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t *s_wave, uint32_t *total) {
    const int w = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (__lane_id() == 63) s_wave[w] = inc;
    __syncthreads();
    uint32_t base = 0;
    for (int k = 0; k < w; k++) base += s_wave[k];
    uint32_t tot = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    __syncthreads();
    if (total) *total = tot;
    return base + inc - v;
}

// Lanes holding the same 8-bit digit (valid lanes only).
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// Block index remap so that consecutive work items land on the same XCD (the dispatcher
// deals workgroups round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
    const uint32_t nx = 8;
    const uint32_t per = nb / nx, rem = nb % nx;
    const uint32_t x = b % nx, k = b / nx;
    // XCD x owns the contiguous range [x*per + min(x, rem), ...) of logical items
    const uint32_t start = x * per + (x < rem ? x : rem);
    const uint32_t cnt = per + (x < rem ? 1 : 0);
    return k < cnt ? start + k : b;  // b beyond the dealt grid cannot happen; keep identity
}

}  // namespace gsr
