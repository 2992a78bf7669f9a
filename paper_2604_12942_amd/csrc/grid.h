// Uniform cell grid over 3-D points, shared by the insertion filter and the loop registration.
// A point's cell is floor(x / cell) per axis (float64); the three cell indices are packed into
// 63 bits (21 each, wrapping) and mixed to a 32-bit hash.  Points are sorted by hash, and a table
// over the hash's top kBucketBits bits narrows a probe to a short binary search.  Distinct cells
// may share a hash: a probe then sees extra candidates, which the caller's exact test rejects.
#pragma once

#include "gsr_internal.h"

namespace gsr {

constexpr int kBucketBits = 16;
constexpr int kBuckets = 1 << kBucketBits;

__device__ __forceinline__ uint32_t cell_hash(int64_t cx, int64_t cy, int64_t cz) {
    uint64_t z = ((uint64_t)cx & 0x1FFFFFull) | (((uint64_t)cy & 0x1FFFFFull) << 21) |
                 (((uint64_t)cz & 0x1FFFFFull) << 42);
    // SplitMix64 finaliser
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (uint32_t)z;
}

__device__ __forceinline__ int64_t cell_of(double x, double inv_cell) { return (int64_t)floor(x * inv_cell); }

// First sorted position of hash h: [lo, hi) from the bucket table, then a binary search.
__device__ __forceinline__ uint32_t grid_lower_bound(const uint32_t *__restrict__ key,
                                                    const uint32_t *__restrict__ bucket, uint32_t h) {
    const uint32_t b = h >> (32 - kBucketBits);
    uint32_t lo = bucket[b], hi = bucket[b + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (key[mid] < h) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Squared distance ((dx dx + dy dy) + dz dz) in float64 with every operation rounded (no
// contraction), so that other implementations can reproduce the decisions exactly.
__device__ __forceinline__ double sqdist_rn(double ax, double ay, double az, double bx, double by, double bz) {
    const double dx = __dsub_rn(ax, bx), dy = __dsub_rn(ay, by), dz = __dsub_rn(az, bz);
    return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

}  // namespace gsr

// Builds the grid over the points means[c * stride + (index ? index[j] : j)], j < count (count
// read on the device when count_dev is given, else cap): keys / vals (= j) sorted by hash, and
// bucket [kBuckets + 1].  k2 / v2 are ping-pong buffers of cap words; sort_ws holds
// gsr_sort_pairs_ws_bytes(cap) bytes.
extern "C" gsr_status gsr_grid_build_launch(const float *means, int64_t stride, const uint32_t *index,
                                            const uint32_t *count_dev, int64_t cap, double cell, uint32_t *keys,
                                            uint32_t *vals, uint32_t *k2, uint32_t *v2, uint32_t *bucket,
                                            void *sort_ws, hipStream_t st);
