// Tile binning: ordered compaction of the visible (view, Gaussian) pairs, a stable LSD radix sort
// of them by float32 depth bits, depth-ordered emission of (view-tile, pair) instances and a
// stable LSD radix sort of the instances by view-tile.  The result equals a lexicographic sort by
// (view, tile, depth bits, Gaussian index) while the expensive instance sort only moves the
// ceil(log2(V*T)) tile bits (two 8-bit passes for up to 65,536 view-tiles) instead of all 47+.
//
// Every kernel reads the live element count from device memory and is launched over the
// capacity, so the whole pipeline runs without a host round-trip (and can be graph-captured).
#include "gsr_internal.h"

namespace gsr {

__device__ __forceinline__ uint32_t dev_count(const uint32_t *n_dev, uint32_t n_host, uint32_t cap) {
    const uint32_t n = n_dev ? *n_dev : n_host;
    return n < cap ? n : cap;
}

// ---- generic helpers -------------------------------------------------------------------------
__global__ void k_copy_u32(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

__global__ void k_fill_u32(uint32_t *__restrict__ dst, uint32_t value, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = value;
}

// Exclusive scan in place of nb (small) block sums by one 1024-thread block; writes the total.
// With lim, only the first ceil(*lim / per) sums are scanned (the rest are zero and unread).
__global__ __launch_bounds__(1024) void k_scan_small(uint32_t *__restrict__ v, int nb, uint32_t *__restrict__ total,
                                                     const uint32_t *__restrict__ lim = nullptr, uint32_t per = 1) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    if (lim) {
        const uint32_t used = (*lim + per - 1) / per;
        nb = used < (uint32_t)nb ? (int)used : nb;
    }
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int idx = base + threadIdx.x;
        const uint32_t x = idx < nb ? v[idx] : 0u;
        uint32_t inc = wave_incl_scan(x);
        const int w = threadIdx.x >> 6;
        if (__lane_id() == 63) s_w[w] = inc;
        __syncthreads();
        uint32_t wb = 0, tot = 0;
        for (int k = 0; k < 16; k++) {
            wb += k < w ? s_w[k] : 0u;
            tot += s_w[k];
        }
        const uint32_t carry = s_carry;
        if (idx < nb) v[idx] = carry + wb + inc - x;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = s_carry;
}

// ---- ordered compaction of visible pairs ---------------------------------------------------------
// Block b covers pairs [b*4096, (b+1)*4096) in round-major order: pair b*4096 + r*256 + t is read by
// thread t in round r, so every load is coalesced; (round, wave, lane) order is pair order.
__global__ __launch_bounds__(256) void k_vis_count(const uint32_t *__restrict__ ntiles, uint32_t VN,
                                                   uint32_t *__restrict__ bsum) {
    __shared__ uint32_t s_w[4];
    const uint32_t base = blockIdx.x * kSortTile;
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t e = base + r * kSortThreads + threadIdx.x;
        c += (e < VN && ntiles[e] > 0) ? 1u : 0u;
    }
    uint32_t tot;
    block_excl_scan256(c, s_w, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_vis_compact(const uint32_t *__restrict__ info, uint32_t VN,
                                                     const uint32_t *__restrict__ boff, uint32_t *__restrict__ keys,
                                                     uint32_t *__restrict__ vals) {
    __shared__ uint32_t s_cnt[kSortItems * 4];
    const uint32_t base = blockIdx.x * kSortTile;
    const int w = threadIdx.x >> 6, lane = __lane_id();
    uint64_t m[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t e = base + r * kSortThreads + threadIdx.x;
        m[r] = __ballot(e < VN && info[e] > 0);
        if (lane == 0) s_cnt[r * 4 + w] = (uint32_t)__popcll(m[r]);
    }
    __syncthreads();
    // exclusive prefix of the 64 (round, wave) counts, in that order
    if (threadIdx.x < kSortItems * 4) {
        const uint32_t c = s_cnt[threadIdx.x];
        s_cnt[threadIdx.x] = wave_incl_scan(c) - c;
    }
    __syncthreads();
    const uint32_t b0 = boff[blockIdx.x];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        if ((m[r] >> lane) & 1ull) {
            const uint32_t e = base + r * kSortThreads + threadIdx.x;
            const uint32_t pos = b0 + s_cnt[r * 4 + w] + (uint32_t)__popcll(m[r] & lt);
            keys[pos] = info[VN + e];
            vals[pos] = e;
        }
    }
}

// ---- exclusive scan of a long uint32 array (the stored-contributor offsets) ------------------
__global__ __launch_bounds__(256) void k_scan_sum(const uint32_t *__restrict__ in, int64_t n,
                                                  uint32_t *__restrict__ bsum) {
    __shared__ uint32_t s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kSortTile + threadIdx.x * kSortItems;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kSortItems; k++) c += base + k < n ? in[base + k] : 0u;
    uint32_t tot;
    block_excl_scan256(c, s_w, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_write(const uint32_t *__restrict__ in, int64_t n,
                                                    const uint32_t *__restrict__ boff, uint32_t *__restrict__ out) {
    __shared__ uint32_t s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kSortTile + threadIdx.x * kSortItems;
    uint32_t x[kSortItems], c = 0;
#pragma unroll
    for (int k = 0; k < kSortItems; k++) {
        x[k] = base + k < n ? in[base + k] : 0u;
        c += x[k];
    }
    uint32_t run = boff[blockIdx.x] + block_excl_scan256(c, s_w, nullptr);
#pragma unroll
    for (int k = 0; k < kSortItems; k++) {
        if (base + k < n) out[base + k] = run;
        run += x[k];
    }
}

// ---- stable LSD radix sort, 8-bit digits -----------------------------------------------------
// Block b sorts items [b*kRadixTile, (b+1)*kRadixTile); the histogram counts each block's digits,
// and the scatter ranks them stably (input order) inside the block.
constexpr int kRadixItems = 12;
constexpr int kRadixTile = kSortThreads * kRadixItems;
__global__ __launch_bounds__(256) void k_radix_hist(const uint32_t *__restrict__ keys, const uint32_t *n_dev,
                                                    uint32_t n_host, uint32_t cap, int shift, int nblocks,
                                                    uint32_t *__restrict__ hist) {
    // Counts are order-free: each thread takes kRadixItems consecutive keys (three 16-byte loads)
    // and adds a run of equal digits to the block's LDS count in one atomic, so nearly sorted
    // input (long runs) costs one add per run and shuffled input one per key.
    __shared__ uint32_t cnt[kRadix];
    const uint32_t n = dev_count(n_dev, n_host, cap);
    // blocks past the live count write nothing: the row scan and the scatter skip them
    if (blockIdx.x * (uint32_t)kRadixTile >= n) return;
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t first = blockIdx.x * kRadixTile + threadIdx.x * kRadixItems;
    if (first < n) {
        uint32_t k[kRadixItems];
        if (first + kRadixItems <= cap && (reinterpret_cast<uintptr_t>(keys) & 15u) == 0) {
#pragma unroll
            for (int q = 0; q < kRadixItems / 4; q++) {
                const uint4 x = *reinterpret_cast<const uint4 *>(keys + first + 4 * q);
                k[4 * q] = x.x, k[4 * q + 1] = x.y, k[4 * q + 2] = x.z, k[4 * q + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int r = 0; r < kRadixItems; r++) k[r] = first + r < cap ? keys[first + r] : 0u;
        }
        const uint32_t m = n - first < (uint32_t)kRadixItems ? n - first : (uint32_t)kRadixItems;
        uint32_t d = (k[0] >> shift) & (kRadix - 1), run = 1;
#pragma unroll
        for (int r = 1; r < kRadixItems; r++) {
            if ((uint32_t)r >= m) break;
            const uint32_t dr = (k[r] >> shift) & (kRadix - 1);
            if (dr != d) {
                atomicAdd(&cnt[d], run);
                d = dr;
                run = 0;
            }
            run++;
        }
        atomicAdd(&cnt[d], run);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Row d of hist (one row per digit, row stride nblocks) is scanned exclusively in place over the
// blocks that hold live items; the row total goes to totals[d].
__global__ __launch_bounds__(256) void k_radix_scan_rows(uint32_t *__restrict__ hist, int nblocks,
                                                         uint32_t *__restrict__ totals, const uint32_t *n_dev,
                                                         uint32_t n_host, uint32_t cap) {
    // one digit's row per workgroup; each thread owns a contiguous run of the row: sum it, one
    // workgroup scan of the run sums, then rewrite the run as exclusive prefixes.  Runs of up to
    // 16 entries (up to 4096 live blocks) stay in registers, loaded all at once.
    __shared__ uint32_t s_w[4];
    uint32_t *row = hist + (int64_t)blockIdx.x * nblocks;
    const uint32_t n = dev_count(n_dev, n_host, cap);
    const int live = (int)((n + kRadixTile - 1) / kRadixTile);
    const int nb = live < nblocks ? live : nblocks;
    const int per = (nb + 255) / 256;
    const int b0 = threadIdx.x * per;
    const int b1 = b0 + per < nb ? b0 + per : nb;
    if (per <= 16) {
        uint32_t x[16];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < 16; k++) {
            x[k] = b0 + k < b1 ? row[b0 + k] : 0u;
            sum += x[k];
        }
        uint32_t tot;
        uint32_t run = block_excl_scan256(sum, s_w, &tot);
#pragma unroll
        for (int k = 0; k < 16; k++) {
            if (b0 + k < b1) row[b0 + k] = run;
            run += x[k];
        }
        if (threadIdx.x == 0) totals[blockIdx.x] = tot;
        return;
    }
    uint32_t sum = 0;
    for (int idx = b0; idx < b1; idx++) sum += row[idx];
    uint32_t tot;
    uint32_t run = block_excl_scan256(sum, s_w, &tot);
    for (int idx = b0; idx < b1; idx++) {
        const uint32_t x = row[idx];
        row[idx] = run;
        run += x;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

// Block b sorts items [b*kRadixTile, (b+1)*kRadixTile): wave w owns the quarter from
// b*kRadixTile + w*kRadixTile/4 on, 64 per round, so (wave, round, lane) order is input order and each wave ranks its items with
// its own running digit counts, without a workgroup barrier per round; the four waves' counts
// then give every digit's local start and each wave's offset inside it.
__global__ __launch_bounds__(256) void k_radix_scatter(const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                       uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                       const uint32_t *__restrict__ vin2, uint32_t *__restrict__ vout2,
                                                       const uint32_t *n_dev, uint32_t n_host, uint32_t cap, int shift,
                                                       int nblocks, const uint32_t *__restrict__ hist,
                                                       const uint32_t *__restrict__ totals) {
    constexpr int kWaveItems = kRadixTile / 4;
    __shared__ uint32_t s_keys[kRadixTile];
    __shared__ uint32_t s_vals[kRadixTile];
    __shared__ uint32_t s_wcnt[4][kRadix];  // per-wave running counts, then per-wave starts
    __shared__ uint32_t s_lstart[kRadix];
    __shared__ uint32_t s_gbase[kRadix];
    __shared__ uint32_t s_w[4];
    const uint32_t n = dev_count(n_dev, n_host, cap);
    const uint32_t base = blockIdx.x * kRadixTile;
    if (base >= n) return;
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    // global start of digit t for this block
    const uint32_t dtot = totals[t];
    const uint32_t dstart = block_excl_scan256(dtot, s_w, nullptr);
    s_gbase[t] = dstart + hist[t * nblocks + blockIdx.x];
    for (int k = 0; k < 4; k++) s_wcnt[k][t] = 0;
    __syncthreads();
    uint32_t mk[kRadixItems], mv[kRadixItems], mrank[kRadixItems], mv2[kRadixItems];
    const uint64_t lt = lanemask_lt();
    const uint32_t wbase = base + w * kWaveItems;
    for (int r = 0; r < kRadixItems; r++) {
        const uint32_t idx = wbase + r * 64 + lane;
        const bool valid = idx < n;
        mk[r] = valid ? kin[idx] : 0u;
        mv[r] = valid ? vin[idx] : 0u;
        mv2[r] = vin2 ? (valid ? vin2[idx] : 0u) : idx;
        const uint32_t d = (mk[r] >> shift) & (kRadix - 1);
        const uint64_t peers = match_digit8(d, valid);
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        // the wave's count of digit d so far (read by every lane before its leader adds)
        const uint32_t before = s_wcnt[w][d];
        mrank[r] = before + rank;
        if (valid && rank == 0) s_wcnt[w][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        const uint32_t c0 = s_wcnt[0][t], c1 = s_wcnt[1][t], c2 = s_wcnt[2][t], c3 = s_wcnt[3][t];
        const uint32_t ls = block_excl_scan256(c0 + c1 + c2 + c3, s_w, nullptr);
        s_lstart[t] = ls;
        s_wcnt[0][t] = ls;
        s_wcnt[1][t] = ls + c0;
        s_wcnt[2][t] = ls + c0 + c1;
        s_wcnt[3][t] = ls + c0 + c1 + c2;
    }
    __syncthreads();
    for (int r = 0; r < kRadixItems; r++) {
        if (wbase + r * 64 + lane < n) {
            const uint32_t p = s_wcnt[w][(mk[r] >> shift) & (kRadix - 1)] + mrank[r];
            s_keys[p] = mk[r];
            s_vals[p] = mv[r];
        }
    }
    __syncthreads();
    const uint32_t bn = (n - base) < (uint32_t)kRadixTile ? (n - base) : (uint32_t)kRadixTile;
    for (int r = 0; r < kRadixItems; r++) {
        const uint32_t p = r * kSortThreads + t;
        if (p < bn) {
            const uint32_t k = s_keys[p];
            const uint32_t d = (k >> shift) & (kRadix - 1);
            const uint32_t dst = s_gbase[d] + (p - s_lstart[d]);
            kout[dst] = k;
            vout[dst] = s_vals[p];
        }
    }
    if (vout2) {
        // the second payload takes the same permutation through the same LDS staging (without
        // vin2 it is each item's input position)
        __syncthreads();
        for (int r = 0; r < kRadixItems; r++) {
            if (wbase + r * 64 + lane < n)
                s_vals[s_wcnt[w][(mk[r] >> shift) & (kRadix - 1)] + mrank[r]] = mv2[r];
        }
        __syncthreads();
        for (int r = 0; r < kRadixItems; r++) {
            const uint32_t p = r * kSortThreads + t;
            if (p < bn) {
                const uint32_t d = (s_keys[p] >> shift) & (kRadix - 1);
                vout2[s_gbase[d] + (p - s_lstart[d])] = s_vals[p];
            }
        }
    }
}

// ---- instance emission in depth order --------------------------------------------------------
// Instance count of each block of 256 depth-ordered visible pairs.
__global__ __launch_bounds__(256) void k_inst_count(const uint32_t *__restrict__ sorted_gid, const uint32_t *n_vis,
                                                    uint32_t cap, const uint32_t *__restrict__ ntiles,
                                                    uint32_t *__restrict__ bsum) {
    __shared__ uint32_t s_w[4];
    const uint32_t n = dev_count(n_vis, 0, cap);
    // blocks of 256 pairs up to the visible count (grid-stride; later sums are never read)
    for (uint32_t b = blockIdx.x; b * 256 < n; b += gridDim.x) {
        const uint32_t idx = b * 256 + threadIdx.x;
        const uint32_t c = idx < n ? ntiles[sorted_gid[idx]] : 0u;
        uint32_t tot;
        block_excl_scan256(c, s_w, &tot);
        if (threadIdx.x == 0) bsum[b] = tot;
    }
}

// Emission of the instances of 256 depth-ordered visible pairs per block, load-balanced: the
// block's instances are spread over its threads (instance k of the block goes to thread
// k mod 256, which finds its pair by binary search over the pairs' offsets in LDS), so the
// writes are coalesced.  A pair's tiles are emitted row-major and consecutively ("emission
// order").  With pair_gid: the emission-ordered list of visible pairs and the emission index of
// each pair's first instance.  (Each instance's emission index is its position here: the sort's
// first pass generates it as the second payload.)
__global__ __launch_bounds__(256) void k_inst_emit(const uint32_t *__restrict__ sorted_gid, const uint32_t *n_vis,
                                                   uint32_t cap_vis, const uint32_t *__restrict__ info, uint32_t VN,
                                                   uint32_t n, uint32_t T, uint32_t ntx,
                                                   const uint32_t *__restrict__ boff, uint32_t *__restrict__ ikey,
                                                   uint32_t *__restrict__ ival,
                                                   uint32_t *__restrict__ pair_gid, uint32_t *__restrict__ pair_first,
                                                   uint32_t cap) {
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_off[256], s_gid[256], s_r0[256], s_r1[256];
    const uint32_t nv = dev_count(n_vis, 0, cap_vis);
    if (blockIdx.x * 256 >= nv) return;
    const uint32_t idx = blockIdx.x * 256 + threadIdx.x;
    const bool valid = idx < nv;
    const uint32_t gid = valid ? sorted_gid[idx] : 0u;
    const uint32_t c = valid ? info[gid] : 0u;
    uint32_t tot;
    const uint32_t excl = block_excl_scan256(c, s_w, &tot);
    const uint32_t base = boff[blockIdx.x];
    s_off[threadIdx.x] = excl;
    s_gid[threadIdx.x] = gid;
    s_r0[threadIdx.x] = valid ? info[2 * VN + gid] : 0u;
    s_r1[threadIdx.x] = valid ? info[3 * VN + gid] : 0u;
    if (valid && pair_gid) {
        pair_gid[idx] = gid;
        pair_first[idx] = base + excl;
    }
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < tot; k += 256) {
        // the last pair whose offset is <= k (pairs without instances share the next one's offset)
        uint32_t lo = 0, hi = 256;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_off[mid] <= k) lo = mid;
            else hi = mid;
        }
        const uint32_t g = s_gid[lo], r0 = s_r0[lo], r1 = s_r1[lo];
        const uint32_t local = k - s_off[lo];
        const uint32_t tx0 = r0 & 0xffffu, ty0 = r0 >> 16, tx1 = r1 & 0xffffu;
        const uint32_t wdt = tx1 - tx0 + 1;
        const uint32_t ly = local / wdt, lx = local - ly * wdt;
        const uint32_t pos = base + k;
        if (pos < cap) {
            ikey[pos] = (g / n) * T + (ty0 + ly) * ntx + tx0 + lx;
            ival[pos] = g;
        }
    }
}

// LPT key of every view-tile, one byte: the instance count as a small float (the exponent
// floor(log2 c) times 16 plus the next four bits below the leading one, so the key grows with the
// count and resolves it to 1/16 of an octave; empty tiles share the key of a single instance,
// counts of 2^16 and more the key of the top step below 2^16), stored as 255 minus that so that an
// ascending stable sort puts the longest tiles first, ties by index.
__device__ __forceinline__ uint32_t lpt_key(uint32_t c) {
    if (c == 0) return 255u;
    const uint32_t e = 31u - (uint32_t)__builtin_clz(c);  // 0 .. 31
    if (e >= 16u) return 0u;
    const uint32_t m = e >= 4u ? (c >> (e - 4u)) & 15u : (c << (4u - e)) & 15u;
    return 255u - (e * 16u + m);
}

__global__ void k_tile_keys(const uint32_t *__restrict__ ranges, uint32_t VT, uint32_t *__restrict__ keys,
                            uint32_t *__restrict__ vals) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < VT; i += gridDim.x * blockDim.x) {
        keys[i] = lpt_key(ranges[2 * i + 1] - ranges[2 * i]);
        vals[i] = i;
    }
}

__global__ void k_tile_ranges(const uint32_t *__restrict__ keys, const uint32_t *n_inst, uint32_t cap,
                              uint32_t *__restrict__ ranges) {
    const uint32_t m = dev_count(n_inst, 0, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const uint32_t k = keys[i];
        if (i == 0 || keys[i - 1] != k) ranges[2 * k] = i;
        if (i + 1 == m || keys[i + 1] != k) ranges[2 * k + 1] = i + 1;
    }
}

// An instance count above the capacity leaves incomplete lists.  Rather than render them, the
// frame is emptied: no pair visible (tile_info row 0 cleared), every tile range empty and no
// emitted pair, so the render, backward, pair sums, projection backward, fused Adam and visible
// list that follow on the stream do nothing.  A no-op when the instances fit.
__global__ void k_overflow_clear(const uint32_t *__restrict__ n_inst, uint32_t cap, uint32_t *__restrict__ ntiles,
                                 uint32_t VN, uint32_t *__restrict__ ranges, uint32_t VT2,
                                 uint32_t *__restrict__ n_pairs) {
    if (*n_inst <= cap) return;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < VN; i += stride) ntiles[i] = 0u;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < VT2; i += stride) ranges[i] = 0u;
    if (n_pairs && blockIdx.x == 0 && threadIdx.x == 0) *n_pairs = 0u;
}

}  // namespace gsr

using namespace gsr;

namespace {

struct BinWs {
    uint32_t *zk0, *zv0, *zk1, *zv1;  // depth sort ping-pong [VN]
    uint32_t *vis_b, *cnt_b;          // block sums [nb_vn], [VN / 256]
    uint32_t *n_vis;                  // 1
    uint32_t *ik0, *ik1, *iv1, *iw1;  // instance sort [cap]
    uint32_t *tk0, *tk1, *tv1;        // tile-order sort [VT]
    uint32_t *hist;                   // [256][max nb]
    uint32_t *totals;                 // [256]
    size_t bytes;
};

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

BinWs layout(void *base, int64_t VN, int64_t cap, int64_t VT) {
    BinWs w{};
    const int64_t nb_vn = ceil_div(VN > 0 ? VN : 1, kSortTile);
    // histogram rows are as long as the largest sort's block count
    int64_t nbm = ceil_div(VN > 0 ? VN : 1, kRadixTile), nbc = ceil_div(cap > 0 ? cap : 1, kRadixTile);
    nbm = nbm > nbc ? nbm : nbc;
    nbc = ceil_div(VT > 0 ? VT : 1, kRadixTile);
    nbm = nbm > nbc ? nbm : nbc;
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t words) {
        uint32_t *r = reinterpret_cast<uint32_t *>(p ? p + off : nullptr);
        off += al(words * 4);
        return r;
    };
    w.zk0 = take(VN); w.zv0 = take(VN); w.zk1 = take(VN); w.zv1 = take(VN);
    w.vis_b = take(nb_vn); w.cnt_b = take(ceil_div(VN > 0 ? VN : 1, 256)); w.n_vis = take(1);
    w.ik0 = take(cap); w.ik1 = take(cap); w.iv1 = take(cap); w.iw1 = take(cap);
    w.tk0 = take(VT); w.tk1 = take(VT); w.tv1 = take(VT);
    w.hist = take((size_t)kRadix * nbm); w.totals = take(kRadix);
    w.bytes = off;
    return w;
}

gsr_status radix_sort(uint32_t *&k, uint32_t *&v, uint32_t *&k2, uint32_t *&v2, const uint32_t *n_dev,
                      uint32_t n_host, uint32_t cap, int bits, uint32_t *hist, uint32_t *totals, hipStream_t st,
                      uint32_t **w = nullptr, uint32_t **w2 = nullptr, bool w_is_position = false) {
    const int nb = (int)ceil_div(cap, kRadixTile);
    for (int shift = 0; shift < bits; shift += kRadixBits) {
        k_radix_hist<<<nb, kSortThreads, 0, st>>>(k, n_dev, n_host, cap, shift, nb, hist);
        k_radix_scan_rows<<<kRadix, 256, 0, st>>>(hist, nb, totals, n_dev, n_host, cap);
        // w_is_position: the second payload starts as each item's input position, generated by
        // the first pass instead of read
        const uint32_t *win = w && !(w_is_position && shift == 0) ? *w : nullptr;
        k_radix_scatter<<<nb, kSortThreads, 0, st>>>(k, v, k2, v2, win, w ? *w2 : nullptr, n_dev,
                                                     n_host, cap, shift, nb, hist, totals);
        uint32_t *tk = k, *tv = v;
        k = k2; v = v2; k2 = tk; v2 = tv;
        if (w) {
            uint32_t *tw = *w;
            *w = *w2;
            *w2 = tw;
        }
    }
    return last_launch();
}

int bit_length(uint64_t x) {
    int b = 0;
    while (x) { b++; x >>= 1; }
    return b;
}

}  // namespace

extern "C" size_t gsr_bin_sort_ws_bytes(int64_t VN, int64_t cap, int64_t VT) { return layout(nullptr, VN, cap, VT).bytes; }

extern "C" gsr_status gsr_bin_sort_launch(uint32_t *info, int64_t n, int V, int ntx, int nty,
                                          uint32_t *inst_gid, const gsr_emission *em, int64_t cap,
                                          uint32_t *ranges, uint32_t *n_inst, uint32_t *tile_order, void *ws,
                                          hipStream_t st) {
    const int64_t VN = (int64_t)V * n;
    const uint32_t T = (uint32_t)(ntx * nty);
    const int64_t VT = (int64_t)V * T;
    BinWs w = layout(ws, VN, cap, VT);
    const int nb_vn = (int)ceil_div(VN > 0 ? VN : 1, kSortTile);
    // 1. ordered compaction of visible pairs: keys = depth bits, values = v*n + i
    k_vis_count<<<nb_vn, 256, 0, st>>>(info, (uint32_t)VN, w.vis_b);
    k_scan_small<<<1, 1024, 0, st>>>(w.vis_b, nb_vn, w.n_vis);
    k_vis_compact<<<nb_vn, 256, 0, st>>>(info, (uint32_t)VN, w.vis_b, w.zk0, w.zv0);
    // 2. stable sort by depth bits (32 bits, 4 passes: result back in zk0 / zv0)
    uint32_t *k = w.zk0, *v = w.zv0, *k2 = w.zk1, *v2 = w.zv1;
    gsr_status s = radix_sort(k, v, k2, v2, w.n_vis, 0, (uint32_t)(VN > 0 ? VN : 1), 32, w.hist, w.totals, st);
    if (s != GSR_OK) return s;
    // 3. instance counts in depth order, scan, emission
    const int nb_p = (int)ceil_div(VN > 0 ? VN : 1, 256);
    k_inst_count<<<nb_p < 4096 ? nb_p : 4096, 256, 0, st>>>(v, w.n_vis, (uint32_t)(VN > 0 ? VN : 1), info, w.cnt_b);
    k_scan_small<<<1, 1024, 0, st>>>(w.cnt_b, nb_p, n_inst, w.n_vis, 256u);
    // the instance sort runs ceil(bits/8) passes; emit into the buffer that makes the last
    // pass land in the sorted-values output (inst_emit when asked for, else inst_gid)
    const int tbits = bit_length((uint64_t)V * T - 1) > 0 ? bit_length((uint64_t)V * T - 1) : 1;
    const int passes = (tbits + kRadixBits - 1) / kRadixBits;
    uint32_t *ek = w.ik0, *ev = (passes % 2 == 0) ? inst_gid : w.iv1;
    uint32_t *ok = w.ik1, *ov = (passes % 2 == 0) ? w.iv1 : inst_gid;
    uint32_t *inst_emit = em ? em->inst_emit : nullptr;
    uint32_t *ew = inst_emit ? ((passes % 2 == 0) ? inst_emit : w.iw1) : nullptr;
    uint32_t *ow = inst_emit ? ((passes % 2 == 0) ? w.iw1 : inst_emit) : nullptr;
    k_inst_emit<<<nb_p, 256, 0, st>>>(v, w.n_vis, (uint32_t)(VN > 0 ? VN : 1), info, (uint32_t)VN, (uint32_t)n, T,
                                      (uint32_t)ntx, w.cnt_b, ek, ev, em ? em->pair_gid : nullptr,
                                      em ? em->pair_first : nullptr, (uint32_t)cap);
    if (em) k_copy_u32<<<1, 64, 0, st>>>(w.n_vis, em->n_pairs, 1);
    // 4. stable sort by view-tile (carrying the emission index along when asked for)
    s = radix_sort(ek, ev, ok, ov, n_inst, 0, (uint32_t)cap, passes * kRadixBits, w.hist, w.totals, st,
                   inst_emit ? &ew : nullptr, inst_emit ? &ow : nullptr, true);
    if (s != GSR_OK) return s;
    // 5. per view-tile [start, end)
    k_fill_u32<<<(int)ceil_div(2 * (int64_t)V * T, 256) < 4096 ? (int)ceil_div(2 * (int64_t)V * T, 256) : 4096, 256, 0,
                 st>>>(ranges, 0u, 2 * (int64_t)V * T);
    const int nr = (int)(ceil_div(cap, 256) < 8192 ? ceil_div(cap, 256) : 8192);
    k_tile_ranges<<<nr, 256, 0, st>>>(ek, n_inst, (uint32_t)cap, ranges);
    k_overflow_clear<<<256, 256, 0, st>>>(n_inst, (uint32_t)cap, info, (uint32_t)VN, ranges, (uint32_t)(2 * VT),
                                          em ? em->n_pairs : nullptr);
    // 6. longest-processing-time order of the view-tiles (descending instance count, to 1/16 of
    // an octave): one 8-bit pass, whose values land in tile_order
    if (tile_order) {
        const int nt = (int)(ceil_div(VT, 256) < 4096 ? ceil_div(VT, 256) : 4096);
        k_tile_keys<<<nt, 256, 0, st>>>(ranges, (uint32_t)VT, w.tk0, w.tv1);
        uint32_t *a = w.tk0, *b = w.tv1, *c = w.tk1, *d = tile_order;
        s = radix_sort(a, b, c, d, nullptr, (uint32_t)VT, (uint32_t)VT, 8, w.hist, w.totals, st);
        if (s != GSR_OK) return s;
    }
    return last_launch();
}

extern "C" gsr_status gsr_fill_u32_launch(void *dst, uint32_t value, int64_t n, hipStream_t st) {
    if (n <= 0) return GSR_OK;
    const int nb = (int)(ceil_div(n, 256) < 8192 ? ceil_div(n, 256) : 8192);
    k_fill_u32<<<nb, 256, 0, st>>>(static_cast<uint32_t *>(dst), value, n);
    return last_launch();
}

__global__ void k_iota_u32(uint32_t *__restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (uint32_t)i;
}

extern "C" gsr_status gsr_tile_order_identity(uint32_t *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return GSR_OK;
    const int nb = (int)(ceil_div(n, 256) < 4096 ? ceil_div(n, 256) : 4096);
    k_iota_u32<<<nb, 256, 0, st>>>(dst, n);
    return last_launch();
}

extern "C" size_t gsr_scan_ws_bytes(int64_t n) { return (size_t)(ceil_div(n > 0 ? n : 1, kSortTile) * 4 + 256); }

// out[i] = sum of in[0..i) (in and out may not alias), *total = sum of all; ws: gsr_scan_ws_bytes.
extern "C" gsr_status gsr_scan_launch(const uint32_t *in, int64_t n, uint32_t *out, uint32_t *total, void *ws,
                                      hipStream_t st) {
    if (n <= 0) return gsr_fill_u32_launch(total, 0u, 1, st);
    const int nb = (int)ceil_div(n, kSortTile);
    uint32_t *bsum = static_cast<uint32_t *>(ws);
    k_scan_sum<<<nb, 256, 0, st>>>(in, n, bsum);
    k_scan_small<<<1, 1024, 0, st>>>(bsum, nb, total);
    k_scan_write<<<nb, 256, 0, st>>>(in, n, bsum, out);
    return last_launch();
}

// Stable LSD radix sort of n (key, value) pairs by the low `bits` key bits (host-side count),
// ping-ponging between (k, v) and (k2, v2): the result is in (k, v) when ceil(bits / 8) is even,
// else in (k2, v2).  ws: gsr_sort_pairs_ws_bytes(n).
extern "C" size_t gsr_sort_pairs_ws_bytes(int64_t n) {
    return (size_t)((int64_t)kRadix * ceil_div(n > 0 ? n : 1, kRadixTile) * 4 + kRadix * 4 + 512);
}

// As gsr_sort_pairs_launch with the count read on the device (*n_dev, at most cap).
extern "C" gsr_status gsr_sort_pairs_dev_launch(uint32_t *k, uint32_t *v, uint32_t *k2, uint32_t *v2,
                                                const uint32_t *n_dev, uint32_t cap, int bits, void *ws,
                                                hipStream_t st) {
    if (cap == 0) return GSR_OK;
    uint32_t *hist = static_cast<uint32_t *>(ws);
    uint32_t *totals = hist + (size_t)kRadix * ceil_div(cap, kRadixTile);
    return radix_sort(k, v, k2, v2, n_dev, cap, cap, bits, hist, totals, st);
}

extern "C" gsr_status gsr_sort_pairs_launch(uint32_t *k, uint32_t *v, uint32_t *k2, uint32_t *v2, uint32_t n, int bits,
                                            void *ws, hipStream_t st) {
    if (n == 0) return GSR_OK;
    uint32_t *hist = static_cast<uint32_t *>(ws);
    uint32_t *totals = hist + (size_t)kRadix * ceil_div(n, kRadixTile);
    return radix_sort(k, v, k2, v2, nullptr, n, n, bits, hist, totals, st);
}

