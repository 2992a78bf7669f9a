// Map maintenance around the optimisation (Sec. III-C): low-opacity pruning under a bounded
// removal ratio, the proximity filter that drops newly initialised Gaussians lying on top of the
// existing map, and the row gather that compacts or appends component-major arrays (parameters
// and their Adam moments travel together).
//
// Pruning is a selection: candidates are compacted in row order, stably radix-sorted on an
// order-preserving encoding of the logit (so equal logits stay in row order), the first
// min(count, budget) are marked, and the survivors are compacted.  Everything stays on the device.
//
// The proximity filter hashes map means into cells of edge slightly above d_min, sorts the 32-bit
// cell hashes, and lets every new mean probe the 27 cells around its own: a hash collision only
// adds candidates, and the exact distance test decides.
#include "grid.h"

extern "C" gsr_status gsr_scan_launch(const uint32_t *, int64_t, uint32_t *, uint32_t *, void *, hipStream_t);
extern "C" size_t gsr_scan_ws_bytes(int64_t);
extern "C" size_t gsr_sort_pairs_ws_bytes(int64_t);
extern "C" gsr_status gsr_sort_pairs_launch(uint32_t *, uint32_t *, uint32_t *, uint32_t *, uint32_t, int, void *,
                                            hipStream_t);
extern "C" gsr_status gsr_sort_pairs_dev_launch(uint32_t *, uint32_t *, uint32_t *, uint32_t *, const uint32_t *,
                                                uint32_t, int, void *, hipStream_t);
extern "C" gsr_status gsr_fill_u32_launch(void *, uint32_t, int64_t, hipStream_t);

namespace gsr {

// Order-preserving map of a float to uint32 (ascending floats give ascending keys).
__device__ __forceinline__ uint32_t float_key(float x) {
    const uint32_t u = __float_as_uint(x);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ void k_prune_flags(const float *__restrict__ logit, const int32_t *__restrict__ seg, int32_t min_seg,
                              int64_t n, float thr, uint32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flag[i] = (logit[i] < thr && (!seg || seg[i] >= min_seg)) ? 1u : 0u;
}

__global__ void k_prune_scatter(const float *__restrict__ logit, const uint32_t *__restrict__ flag,
                                const uint32_t *__restrict__ off, int64_t n, uint32_t *__restrict__ key,
                                uint32_t *__restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    key[off[i]] = float_key(logit[i]);
    val[off[i]] = (uint32_t)i;
}

// keep[i] = 0 for the first min(count, budget) sorted candidates (keep was filled with 1)
__global__ void k_prune_mark(const uint32_t *__restrict__ sorted_val, const uint32_t *__restrict__ count,
                             uint64_t budget, uint32_t *__restrict__ keep) {
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t c = *count;
    if (j < c && j < budget) keep[sorted_val[j]] = 0u;
}

// out[off[i]] = i for every flagged i (ordered compaction of row indices)
__global__ void k_compact_index(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ off, int64_t n,
                                uint32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) out[off[i]] = (uint32_t)i;
}

struct RowGroupsDev {
    const uint32_t *src[GSR_MAX_ROW_GROUPS];
    uint32_t *dst[GSR_MAX_ROW_GROUPS];
    int32_t col_end[GSR_MAX_ROW_GROUPS];  // exclusive running column count
    int32_t n_groups;
};

constexpr int kGatherCols = 8;  // columns per block: the row index is read once for all of them

// dst[c][dst_offset + j] = src[c][index ? index[j] : j]; blockIdx.y walks chunks of kGatherCols
// consecutive columns of the groups' concatenated column list
__global__ __launch_bounds__(256) void k_gather_rows(RowGroupsDev G, int total_cols, int64_t src_rows,
                                                     const uint32_t *__restrict__ index, int64_t n_rows,
                                                     int64_t dst_rows, int64_t dst_offset) {
    const int col0 = blockIdx.y * kGatherCols;
    const uint32_t *s[kGatherCols];
    uint32_t *d[kGatherCols];
    int g = 0;
#pragma unroll
    for (int q = 0; q < kGatherCols; q++) {
        const int col = col0 + q < total_cols ? col0 + q : total_cols - 1;
        while (g + 1 < G.n_groups && col >= G.col_end[g]) g++;
        const int c = col - (g ? G.col_end[g - 1] : 0);
        s[q] = G.src[g] + (int64_t)c * src_rows;
        d[q] = G.dst[g] + (int64_t)c * dst_rows + dst_offset;
    }
    const int nq = total_cols - col0 < kGatherCols ? total_cols - col0 : kGatherCols;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n_rows; j += (int64_t)gridDim.x * 256) {
        const int64_t r = index ? (int64_t)index[j] : j;
        if (r >= src_rows) continue;
        uint32_t x[kGatherCols];
#pragma unroll
        for (int q = 0; q < kGatherCols; q++) x[q] = q < nq ? s[q][r] : 0u;
#pragma unroll
        for (int q = 0; q < kGatherCols; q++)
            if (q < nq) d[q][j] = x[q];
    }
}

// ---- grid over points (the insertion filter's map, the registration's target set) -------------
__global__ void k_grid_cells(const float *__restrict__ means, int64_t stride, const uint32_t *__restrict__ index,
                             const uint32_t *__restrict__ count_dev, int64_t cap, double inv_cell,
                             uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = count_dev ? (int64_t)*count_dev : cap;
    if (j >= n || j >= cap) return;
    const int64_t i = index ? (int64_t)index[j] : j;
    key[j] = cell_hash(cell_of(means[i], inv_cell), cell_of(means[stride + i], inv_cell),
                       cell_of(means[2 * stride + i], inv_cell));
    val[j] = (uint32_t)j;
}

// bucket[b] = first sorted position whose hash has top bits >= b; bucket[kBuckets] = count
__global__ void k_bucket_bounds(const uint32_t *__restrict__ key, const uint32_t *__restrict__ count_dev, int64_t cap,
                                uint32_t *__restrict__ bucket) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > kBuckets) return;
    int64_t n = count_dev ? (int64_t)*count_dev : cap;
    n = n < cap ? n : cap;
    if (b == kBuckets) {
        bucket[b] = (uint32_t)n;
        return;
    }
    const uint32_t target = (uint32_t)b << (32 - kBucketBits);
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    bucket[b] = (uint32_t)lo;
}

__global__ __launch_bounds__(256) void k_proximity(const float *__restrict__ map, int64_t n_map,
                                                   const float *__restrict__ nw, int64_t n_new, double inv_cell,
                                                   double dd, const uint32_t *__restrict__ key,
                                                   const uint32_t *__restrict__ val, const uint32_t *__restrict__ bucket,
                                                   uint8_t *__restrict__ keep, uint32_t *__restrict__ flag) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_new) return;
    const double px = nw[j], py = nw[n_new + j], pz = nw[2 * n_new + j];
    const int64_t cx = cell_of(px, inv_cell), cy = cell_of(py, inv_cell), cz = cell_of(pz, inv_cell);
    bool found = false;
    for (int d = 0; d < 27 && !found; d++) {
        const uint32_t h = cell_hash(cx + d % 3 - 1, cy + (d / 3) % 3 - 1, cz + d / 9 - 1);
        for (uint32_t e = grid_lower_bound(key, bucket, h); e < (uint32_t)n_map && key[e] == h && !found; e++) {
            const uint32_t i = val[e];
            // ((dx dx + dy dy) + dz dz) < d_min^2 in float64
            found = sqdist_rn(px, py, pz, map[i], map[n_map + i], map[2 * n_map + i]) < dd;
        }
    }
    keep[j] = found ? 0 : 1;
    flag[j] = found ? 0u : 1u;
}

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

struct PruneWs {
    uint32_t *flag, *off, *k, *v, *k2, *v2, *count;
    void *scan, *sort;
    size_t bytes;
};

PruneWs prune_layout(void *base, int64_t n) {
    PruneWs w;
    const size_t words = a256((size_t)(n > 0 ? n : 1) * 4);
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t b) {
        void *r = p ? p + off : nullptr;
        off += a256(b);
        return r;
    };
    w.flag = (uint32_t *)take(words);
    w.off = (uint32_t *)take(words);
    w.k = (uint32_t *)take(words);
    w.v = (uint32_t *)take(words);
    w.k2 = (uint32_t *)take(words);
    w.v2 = (uint32_t *)take(words);
    w.count = (uint32_t *)take(256);
    w.scan = take(gsr_scan_ws_bytes(n));
    w.sort = take(gsr_sort_pairs_ws_bytes(n));
    w.bytes = off;
    return w;
}

struct ProxWs {
    uint32_t *k, *v, *k2, *v2, *bucket, *flag, *off;
    void *scan, *sort;
    size_t bytes;
};

ProxWs prox_layout(void *base, int64_t n_map, int64_t n_new) {
    ProxWs w;
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t b) {
        void *r = p ? p + off : nullptr;
        off += a256(b);
        return r;
    };
    const size_t wm = (size_t)(n_map > 0 ? n_map : 1) * 4, wn = (size_t)(n_new > 0 ? n_new : 1) * 4;
    w.k = (uint32_t *)take(wm);
    w.v = (uint32_t *)take(wm);
    w.k2 = (uint32_t *)take(wm);
    w.v2 = (uint32_t *)take(wm);
    w.bucket = (uint32_t *)take((size_t)(kBuckets + 1) * 4);
    w.flag = (uint32_t *)take(wn);
    w.off = (uint32_t *)take(wn);
    w.scan = take(gsr_scan_ws_bytes(n_new));
    w.sort = take(gsr_sort_pairs_ws_bytes(n_map));
    w.bytes = off;
    return w;
}

// ---- row order: segment-major, Morton order of the means within a segment --------------------
constexpr int kBoxBlocks = 256;

// Per-block minimum and maximum of each coordinate: part[b][0..2] = min, part[b][3..5] = max.
__global__ __launch_bounds__(256) void k_box_part(const float *__restrict__ means, int64_t n,
                                                  float *__restrict__ part) {
    float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int a = 0; a < 3; a++) {
            const float x = means[a * n + i];
            lo[a] = fminf(lo[a], x);
            hi[a] = fmaxf(hi[a], x);
        }
    __shared__ float s[6][256];
    for (int a = 0; a < 3; a++) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int a = 0; a < 3; a++) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + h]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + h]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// Spread the low 10 bits of x to every third bit.
__device__ __forceinline__ uint32_t spread3(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// box[0..2] = minimum, box[3..5] = maximum over the per-block partials.
__global__ void k_box_final(const float *__restrict__ part, int nparts, float *__restrict__ box) {
    if (threadIdx.x >= 6) return;
    const int a = threadIdx.x;
    float r = a < 3 ? 3.0e38f : -3.0e38f;
    for (int b = 0; b < nparts; b++) r = a < 3 ? fminf(r, part[b * 6 + a]) : fmaxf(r, part[b * 6 + a]);
    box[a] = r;
}

// key[i] = Morton code of the mean's cell on a 1024^3 grid over the box (x bits lowest), val[i] = i.
// The cell is floor((x - lo) * (1024 / (hi - lo))) in float32, clamped to [0, 1023].
__global__ void k_morton_keys(const float *__restrict__ means, int64_t n, const float *__restrict__ box,
                              uint32_t *__restrict__ key, uint32_t *__restrict__ val) {
    float lo[3], sc[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = box[a];
        sc[a] = box[3 + a] > box[a] ? 1024.0f / (box[3 + a] - box[a]) : 0.0f;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t k = 0;
        for (int a = 0; a < 3; a++) {
            const float c = floorf((means[a * n + i] - lo[a]) * sc[a]);
            const uint32_t q = c >= 1023.0f ? 1023u : (c > 0.0f ? (uint32_t)c : 0u);
            k |= spread3(q) << a;
        }
        key[i] = k;
        val[i] = (uint32_t)i;
    }
}

// key[j] = segment of row order[j], sign bit flipped so that the unsigned order is the signed one.
__global__ void k_segment_keys(const int32_t *__restrict__ seg, const uint32_t *__restrict__ order, int64_t n,
                               uint32_t *__restrict__ key) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        key[j] = (uint32_t)seg[order[j]] ^ 0x80000000u;
}

struct OrderWs {
    float *part;
    uint32_t *key, *k2, *v2;
    void *sort;
    size_t bytes;
};

OrderWs order_layout(void *base, int64_t n) {
    OrderWs w{};
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t b) {
        void *r = p ? p + off : nullptr;
        off += a256(b);
        return r;
    };
    const size_t wn = (size_t)(n > 0 ? n : 1) * 4;
    w.part = (float *)take((size_t)(kBoxBlocks + 1) * 6 * 4);  // partials, then the box
    w.key = (uint32_t *)take(wn);
    w.k2 = (uint32_t *)take(wn);
    w.v2 = (uint32_t *)take(wn);
    w.sort = take(gsr_sort_pairs_ws_bytes(n));
    w.bytes = off;
    return w;
}

int nblk(int64_t n) { return (int)ceil_div(n > 0 ? n : 1, 256); }

}  // namespace gsr

using namespace gsr;

extern "C" gsr_status gsr_grid_build_launch(const float *means, int64_t stride, const uint32_t *index,
                                            const uint32_t *count_dev, int64_t cap, double cell, uint32_t *keys,
                                            uint32_t *vals, uint32_t *k2, uint32_t *v2, uint32_t *bucket,
                                            void *sort_ws, hipStream_t st) {
    if (cap > 0) {
        k_grid_cells<<<nblk(cap), 256, 0, st>>>(means, stride, index, count_dev, cap, 1.0 / cell, keys, vals);
        gsr_status s = count_dev
                           ? gsr_sort_pairs_dev_launch(keys, vals, k2, v2, count_dev, (uint32_t)cap, 32, sort_ws, st)
                           : gsr_sort_pairs_launch(keys, vals, k2, v2, (uint32_t)cap, 32, sort_ws, st);
        if (s != GSR_OK) return s;
    }
    k_bucket_bounds<<<nblk(kBuckets + 1), 256, 0, st>>>(keys, count_dev, cap, bucket);
    return last_launch();
}

extern "C" size_t gsr_prune_ws_bytes(int64_t n) { return prune_layout(nullptr, n).bytes; }

extern "C" gsr_status gsr_prune_launch(const float *logit, const int32_t *seg, int32_t min_seg, int64_t n, float thr,
                                       uint64_t budget, uint32_t *keep_index, uint32_t *n_keep, void *ws,
                                       hipStream_t st) {
    if (n == 0) return gsr_fill_u32_launch(n_keep, 0u, 1, st);
    PruneWs w = prune_layout(ws, n);
    k_prune_flags<<<nblk(n), 256, 0, st>>>(logit, seg, min_seg, n, thr, w.flag);
    gsr_status s = gsr_scan_launch(w.flag, n, w.off, w.count, w.scan, st);
    if (s != GSR_OK) return s;
    k_prune_scatter<<<nblk(n), 256, 0, st>>>(logit, w.flag, w.off, n, w.k, w.v);
    // four 8-bit passes: the sorted pairs end in (k, v)
    s = gsr_sort_pairs_dev_launch(w.k, w.v, w.k2, w.v2, w.count, (uint32_t)n, 32, w.sort, st);
    if (s != GSR_OK) return s;
    s = gsr_fill_u32_launch(w.flag, 1u, n, st);  // flag becomes the keep flag
    if (s != GSR_OK) return s;
    if (budget > 0) k_prune_mark<<<nblk(n), 256, 0, st>>>(w.v, w.count, budget, w.flag);
    s = gsr_scan_launch(w.flag, n, w.off, n_keep, w.scan, st);
    if (s != GSR_OK) return s;
    k_compact_index<<<nblk(n), 256, 0, st>>>(w.flag, w.off, n, keep_index);
    return last_launch();
}

extern "C" gsr_status gsr_gather_launch(const gsr_row_groups *g, int64_t src_rows, const uint32_t *index,
                                        int64_t n_rows, int64_t dst_rows, int64_t dst_offset, hipStream_t st) {
    RowGroupsDev G;
    int cols = 0;
    for (int k = 0; k < g->n_groups; k++) {
        G.src[k] = static_cast<const uint32_t *>(g->src[k]);
        G.dst[k] = static_cast<uint32_t *>(g->dst[k]);
        cols += g->cols[k];
        G.col_end[k] = cols;
    }
    G.n_groups = g->n_groups;
    if (n_rows == 0 || cols == 0) return GSR_OK;
    const int nbx = (int)(ceil_div(n_rows, 256) < 512 ? ceil_div(n_rows, 256) : 512);
    k_gather_rows<<<dim3(nbx, (unsigned)ceil_div(cols, kGatherCols)), 256, 0, st>>>(G, cols, src_rows, index, n_rows,
                                                                                    dst_rows, dst_offset);
    return last_launch();
}

extern "C" size_t gsr_proximity_ws_bytes(int64_t n_map, int64_t n_new) { return prox_layout(nullptr, n_map, n_new).bytes; }

extern "C" gsr_status gsr_proximity_launch(const float *map, int64_t n_map, const float *nw, int64_t n_new, float d_min,
                                           uint8_t *keep, uint32_t *keep_index, uint32_t *n_keep, void *ws,
                                           hipStream_t st) {
    if (n_new == 0) return gsr_fill_u32_launch(n_keep, 0u, 1, st);
    ProxWs w = prox_layout(ws, n_map, n_new);
    // cells a little wider than d_min: two means closer than d_min always fall in neighbouring
    // cells even after the float64 rounding of x / cell
    const double cell = (double)d_min * (1.0 + 1.0 / (1 << 20));
    const double inv_cell = 1.0 / cell;
    const double dd = (double)d_min * (double)d_min;
    gsr_status s = gsr_grid_build_launch(map, n_map, nullptr, nullptr, n_map, cell, w.k, w.v, w.k2, w.v2, w.bucket,
                                         w.sort, st);
    if (s != GSR_OK) return s;
    k_proximity<<<nblk(n_new), 256, 0, st>>>(map, n_map, nw, n_new, inv_cell, dd, w.k, w.v, w.bucket, keep, w.flag);
    s = gsr_scan_launch(w.flag, n_new, w.off, n_keep, w.scan, st);
    if (s != GSR_OK) return s;
    k_compact_index<<<nblk(n_new), 256, 0, st>>>(w.flag, w.off, n_new, keep_index);
    return last_launch();
}

extern "C" size_t gsr_row_order_ws_bytes(int64_t n) { return order_layout(nullptr, n).bytes; }

// order[j] = the row that moves to position j: rows by segment id (when given), then by the Morton
// code of the mean, ties by row index (both sorts are stable).
extern "C" gsr_status gsr_row_order_launch(const float *means, const int32_t *seg, int64_t n, uint32_t *order,
                                           void *ws, hipStream_t st) {
    if (n == 0) return GSR_OK;
    OrderWs w = order_layout(ws, n);
    const int nb = (int)(ceil_div(n, 256) < kBoxBlocks ? ceil_div(n, 256) : kBoxBlocks);
    k_box_part<<<nb, 256, 0, st>>>(means, n, w.part);
    const int ng = (int)(ceil_div(n, 256) < 4096 ? ceil_div(n, 256) : 4096);
    float *box = w.part + kBoxBlocks * 6;
    k_box_final<<<1, 64, 0, st>>>(w.part, nb, box);
    k_morton_keys<<<ng, 256, 0, st>>>(means, n, box, w.key, order);
    // four 8-bit passes each: the sorted pairs end in (key, order)
    gsr_status s = gsr_sort_pairs_launch(w.key, order, w.k2, w.v2, (uint32_t)n, 32, w.sort, st);
    if (s != GSR_OK || !seg) return s;
    k_segment_keys<<<ng, 256, 0, st>>>(seg, order, n, w.key);
    return gsr_sort_pairs_launch(w.key, order, w.k2, w.v2, (uint32_t)n, 32, w.sort, st);
}
