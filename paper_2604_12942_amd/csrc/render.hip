// Front-to-back alpha compositing of colour and depth (Eq. 8) and its exact backward.
//
// One 256-lane workgroup (four wave64s) per (view, screen tile); one pixel per lane, so each
// wave owns a sub-rectangle of the tile (16x4, 8x8 or 32x2 pixels).  Workgroups are launched in
// longest-list-first order.  The tile's depth-ordered instances are staged through LDS in batches
// of 256: each lane gathers one projected splat (48 B), re-centres its double-precision mean on
// the 32x32-aligned block that holds the tile, and stores the float32 fields the blend loop needs.
// Each wave then tests every staged Gaussian's alpha >= 1/255 ellipse against its own pixel
// sub-rectangle (exact minimum of the quadratic form over the rectangle) and walks only the
// Gaussians that reach it.  The blend exponent is the whitened form |L^T D|^2 (L the Cholesky
// factor of (log2(e)/2) Q): no cancellation for thin ellipses; exp2 is the hardware v_exp_f32.
#include <type_traits>

#include "gsr_internal.h"

namespace gsr {

// Staged splat (LDS): A = (mx, my, l11, l21), B = (l22, cut = log2(255 o), o, z), C = (r, g, b, -)
__device__ __forceinline__ void stage_splat(const gsr_splat *__restrict__ splats, uint32_t gid, double ox, double oy,
                                            float4 &A, float4 &B, float4 &C) {
    const double2 uv = *reinterpret_cast<const double2 *>(splats + gid);
    const float4 f1 = *(reinterpret_cast<const float4 *>(splats + gid) + 1);
    const float4 f2 = *(reinterpret_cast<const float4 *>(splats + gid) + 2);
    A = make_float4((float)(uv.x - ox), (float)(uv.y - oy), f1.x, f1.y);
    B = make_float4(f1.z, __log2f(255.0f * f1.w), f1.w, f2.x);
    C = make_float4(f2.y, f2.z, f2.w, 0.0f);
}

// Whitened exponent at the pixel centre (fx, fy) (32x32-block coordinates).  The forward calls
// this and the backward performs the same operations on the same operands, so their contribute /
// skip decisions are bit-identical.
__device__ __forceinline__ float blend_exponent(const float4 &A, float l22, float fx, float fy, float &dx, float &dy,
                                                float &u1, float &u2) {
    dx = fx - A.x;
    dy = fy - A.y;
    u1 = __builtin_fmaf(A.z, dx, A.w * dy);
    u2 = l22 * dy;
    return __builtin_fmaf(u1, u1, u2 * u2);
}

// Does the ellipse |L^T (p - m)|^2 <= cut reach the box [x0, x1] x [y0, y1] of pixel centres?
// The minimum of the convex quadratic over the box is 0 if the mean is inside, else it lies on
// an edge, where the restriction is a 1-D quadratic minimised by clamping.  The small margin
// keeps the test conservative against the float32 rounding of the per-pixel evaluation.
__device__ __forceinline__ bool ellipse_meets_box(const float4 &A, const float4 &B, float x0, float x1, float y0,
                                                  float y1) {
    const float ax = x0 - A.x, bx = x1 - A.x, ay = y0 - A.y, by = y1 - A.y;
    if (ax <= 0.f && bx >= 0.f && ay <= 0.f && by >= 0.f) return true;
    const float l11 = A.z, l21 = A.w, l22 = B.x;
    const float q = l21 * l21 + l22 * l22;
    float best = 3.0e38f;
    {   // vertical edges: dx fixed, minimise over dy
        const float dys0 = fminf(fmaxf(-(l11 * l21 * ax) / q, ay), by);
        const float u0 = l11 * ax + l21 * dys0, v0 = l22 * dys0;
        best = fminf(best, u0 * u0 + v0 * v0);
        const float dys1 = fminf(fmaxf(-(l11 * l21 * bx) / q, ay), by);
        const float u1 = l11 * bx + l21 * dys1, v1 = l22 * dys1;
        best = fminf(best, u1 * u1 + v1 * v1);
    }
    {   // horizontal edges: dy fixed, minimise over dx
        const float dxs0 = fminf(fmaxf(-(l21 * ay) / l11, ax), bx);
        const float u0 = l11 * dxs0 + l21 * ay, v0 = l22 * ay;
        best = fminf(best, u0 * u0 + v0 * v0);
        const float dxs1 = fminf(fmaxf(-(l21 * by) / l11, ax), bx);
        const float u1 = l11 * dxs1 + l21 * by, v1 = l22 * by;
        best = fminf(best, u1 * u1 + v1 * v1);
    }
    return best <= B.y * 1.001f + 1e-3f;
}

// Pixel-centre box of the wave's 64 pixels in 32x32-block coordinates.
template <int TW>
__device__ __forceinline__ void wave_box(int tx0, int ty0, int w, float &x0, float &x1, float &y0, float &y1) {
    constexpr int rows = 64 / TW;
    x0 = (float)tx0 + 0.5f;
    x1 = (float)(tx0 + TW - 1) + 0.5f;
    y0 = (float)(ty0 + w * rows) + 0.5f;
    y1 = (float)(ty0 + w * rows + rows - 1) + 0.5f;
}

// ---- front-to-back walk -----------------------------------------------------------------------
constexpr int kNullSlot = 256;    // LDS slot of the null Gaussian (cut-off below every exponent)
constexpr float kGone = 1.0e30f;  // centre of a finished pixel: out of reach of every ellipse

// The calling lane's pixel in one (view, tile) work item.
struct TileGeom {
    int v, px, py;
    bool inside;
    double ox, oy;             // origin of the 32x32-aligned block holding the tile
    float fx, fy;              // pixel centre in block coordinates
    float wx0, wx1, wy0, wy1;  // the wave's box of pixel centres
};

template <int TW, int TH>
__device__ __forceinline__ TileGeom tile_geom(uint32_t item, int T, int ntx, int W, int H) {
    TileGeom t;
    t.v = item / T;
    const int tile = item % T;
    const int tx = tile % ntx, ty = tile / ntx;
    t.px = tx * TW + (int)threadIdx.x % TW;
    t.py = ty * TH + (int)threadIdx.x / TW;
    t.inside = t.px < W && t.py < H;
    // means are re-centred on the 32x32-aligned block holding the tile: the same origin for
    // every tile shape, so whole-tile images are bit-identical across 16x16, 8x32 and 32x8 tiles
    const int bx = (tx * TW) & ~31, by = (ty * TH) & ~31;
    t.ox = (double)bx;
    t.oy = (double)by;
    t.fx = (float)(t.px - bx) + 0.5f;
    t.fy = (float)(t.py - by) + 0.5f;
    wave_box<TW>(tx * TW - bx, ty * TH - by, (int)threadIdx.x >> 6, t.wx0, t.wx1, t.wy0, t.wy1);
    return t;
}

// Per-pixel state of the walk.  A finished pixel (terminated, or outside the image) moves its
// centre to kGone: the exponent then overflows to +inf, the pixel blends with weight 0, and the
// loop needs no separate flag.
struct PixelWalk {
    float Tr, c0, c1, c2, dd;
    uint32_t lst, nc;
    float fxl;
};

__device__ __forceinline__ PixelWalk walk_start(const TileGeom &t, float T0) {
    PixelWalk w;
    w.Tr = T0;
    w.c0 = w.c1 = w.c2 = w.dd = 0.f;
    w.lst = w.nc = 0;
    w.fxl = (t.inside && T0 >= GSR_T_MIN) ? t.fx : kGone;
    return w;
}

// Composites the instances [lo, hi) of a tile list that begins at `start` (positions count from
// it) into the walk.  The instances are staged through LDS in batches of 256; each wave tests
// every staged ellipse against its pixel box and walks only the Gaussians that reach it, two per
// step (the second one's LDS reads are in flight during the first blend; an odd last one is
// paired with the null slot).  A wave stops at the first step after which all its pixels have
// finished, the workgroup at the first batch none of its pixels needs.  Block-uniform arguments;
// the null slot must have been written before the call.
// What a walk keeps besides the transmittance and the termination, from least to most: nothing
// (the depth slices' transmittance products), the colour, depth and last contributor (an image),
// also the number of contributors, or also (the second pass of the stored-contributor mode) the
// tile-list positions of the composited Gaussians, front to back, at clist[cbase ...] (skipped
// beyond ccap).
enum WalkKeeps : int { kKeepTrans = 0, kKeepImage = 1, kKeepCount = 2, kKeepStore = 3 };

template <int KEEP>
__device__ __forceinline__ void composite(const gsr_splat *__restrict__ splats, const uint32_t *__restrict__ inst,
                                          uint32_t start, uint32_t lo, uint32_t hi, const TileGeom &t,
                                          float4 *sA, float4 *sB, float4 *sC, PixelWalk &pw,
                                          uint32_t *__restrict__ clist, uint32_t cbase, uint32_t ccap) {
    for (uint32_t b = lo; b < hi; b += 256) {
        if (__syncthreads_count(pw.fxl != kGone) == 0) break;
        const uint32_t e = b + threadIdx.x;
        const int cnt = (int)min(256u, hi - b);
        if (e < hi) {
            float4 A, B, C;
            stage_splat(splats, inst[e], t.ox, t.oy, A, B, C);
            sA[threadIdx.x] = A;
            sB[threadIdx.x] = B;
            sC[threadIdx.x] = C;
        }
        __syncthreads();
        const uint32_t pos0 = b - start + 1;
        // one Gaussian's blend into this lane's pixel (branch-free: a non-contributing lane
        // blends with weight exactly 0)
        auto blend = [&](int j, const float4 &A, const float4 &B, const float4 &C) {
            float dx, dy, u1, u2;
            const float P = blend_exponent(A, B.x, pw.fxl, t.fy, dx, dy, u1, u2);
            const bool cont = P <= B.y;
            const float ar = B.z * __builtin_amdgcn_exp2f(-P);
            const float a0 = cont ? fminf(ar, GSR_ALPHA_MAX) : 0.0f;
            const float Tn = pw.Tr * (1.0f - a0);
            const bool term = Tn < GSR_T_MIN;
            pw.fxl = term ? kGone : pw.fxl;
            const float a = term ? 0.0f : a0;
            if constexpr (KEEP >= kKeepImage) {
                const float wgt = a * pw.Tr;
                pw.c0 = __builtin_fmaf(wgt, C.x, pw.c0);
                pw.c1 = __builtin_fmaf(wgt, C.y, pw.c1);
                pw.c2 = __builtin_fmaf(wgt, C.z, pw.c2);
                pw.dd = __builtin_fmaf(wgt, B.w, pw.dd);
            }
            pw.Tr = term ? pw.Tr : Tn;
            if constexpr (KEEP >= kKeepImage) {
                const bool used = a > 0.0f;
                if (KEEP == kKeepStore && used && cbase + pw.nc < ccap) clist[cbase + pw.nc] = pos0 - 1 + (uint32_t)j;
                pw.lst = used ? pos0 + (uint32_t)j : pw.lst;
                if constexpr (KEEP >= kKeepCount) pw.nc += used ? 1u : 0u;
            }
        };
        for (int g = 0; g < 4 && g * 64 < cnt; g++) {
            if (__ballot(pw.fxl != kGone) == 0) break;
            const int slot = g * 64 + __lane_id();
            const bool r = slot < cnt && ellipse_meets_box(sA[slot], sB[slot], t.wx0, t.wx1, t.wy0, t.wy1);
            uint64_t m = __ballot(r);
            while (m) {
                const int j1 = g * 64 + __builtin_ctzll(m);
                m &= m - 1;
                const int j2 = m ? g * 64 + __builtin_ctzll(m) : kNullSlot;
                m &= m - 1;
                const float4 A1 = sA[j1], B1 = sB[j1], C1 = sC[j1];
                const float4 A2 = sA[j2], B2 = sB[j2], C2 = sC[j2];
                blend(j1, A1, B1, C1);
                blend(j2, A2, B2, C2);
                if (__ballot(pw.fxl != kGone) == 0) break;
            }
        }
    }
}

__device__ __forceinline__ void write_null_slot(float4 *sA, float4 *sB, float4 *sC) {
    if (threadIdx.x == 0) {
        sA[kNullSlot] = make_float4(0.f, 0.f, 0.f, 0.f);
        sB[kNullSlot] = make_float4(0.f, -1.f, 0.f, 0.f);
        sC[kNullSlot] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

// ---- depth slices of long tiles ------------------------------------------------------------------
// A tile whose list holds tens of thousands of instances would keep one workgroup busy long after
// the rest of the launch has drained (a view down a corridor piles them into the tile at the
// vanishing point).  A tile longer than kSplitMin is cut into slices of kSliceLen consecutive
// instances.  Compositing is associative in the transmittance: the walk through
// slice k starts from T_in(k), the product over the earlier slices of their own (1 - a)
// products, and the pixel has terminated before slice k exactly when T_in(k) < 1e-4 (T never
// increases).  So one pass computes every slice's product (as the product of its sub-slices'
// products; a pixel whose product over a sub-slice falls below 1e-4 stops and records 0, which
// can only happen when it terminates there), a second composites all slices at once from their
// T_in, and a merge sums each pixel's slice results in order, stopping after the slice in which
// it terminated.  The results are those of the whole-tile walk up to the float rounding of the
// transmittance products (which are associated per sub-slice).
constexpr uint32_t kSliceLen = 1024;
constexpr uint32_t kSplitMin = 8 * kSliceLen;  // shorter tiles finish within the launch anyway
// The product pass walks each slice as kSubs sub-slices of kSubLen instances (one LDS batch each)
// in separate workgroups: shorter walks, spread over more workgroups.
constexpr uint32_t kSubLen = 256;
constexpr uint32_t kSubs = kSliceLen / kSubLen;
constexpr uint32_t kNoSlice = 0xffffffffu;  // list entry of a slice that did not fit

struct SliceArgs {
    const uint32_t *tile_slices;  // [V*T] number of slices of each view-tile (0: whole tile)
    const uint2 *info;            // [cap] (view-tile, slice index within the tile)
    const uint32_t *count;        // [1] number of slices
    float *tprod;                 // [cap][kSubs][256] per-pixel product of (1 - a) over each sub-slice
    float4 *part;                 // [cap][256] slice colour (3) and depth, already times T_in
    uint2 *part2;                 // [cap][256] (T after the slice, negated if it terminated there;
                                  //             last composited position)
    uint32_t cap, grid;           // slice capacity; workgroups that walk the slice list
};

__global__ void k_slice_count(const uint32_t *__restrict__ ranges, uint32_t VT, uint32_t *__restrict__ ns) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < VT; i += gridDim.x * blockDim.x) {
        const uint32_t len = ranges[2 * i + 1] - ranges[2 * i];
        ns[i] = len > kSplitMin ? (len + kSliceLen - 1) / kSliceLen : 0u;
    }
}

// Lists the slices tile by tile.  A tile whose slices would not fit the capacity (impossible
// while the lists hold at most the capacity the slice list was sized for) is left whole.
__global__ void k_slice_emit(uint32_t *__restrict__ ns, const uint32_t *__restrict__ off, uint32_t VT,
                             uint32_t cap, uint2 *__restrict__ info) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < VT; i += gridDim.x * blockDim.x) {
        const uint32_t k = ns[i];
        if (!k) continue;
        if (off[i] + k > cap) {
            ns[i] = 0;
            for (uint32_t q = off[i]; q < cap && q < off[i] + k; q++) info[q] = make_uint2(kNoSlice, 0u);
            continue;
        }
        for (uint32_t q = 0; q < k; q++) info[off[i] + q] = make_uint2(i, q);
    }
}

// This pixel's product of (1 - a) over slice j, in sub-slice order.
__device__ __forceinline__ float slice_prod(const SliceArgs &sl, uint32_t j) {
    float P = 1.0f;
#pragma unroll
    for (uint32_t u = 0; u < kSubs; u++) P *= sl.tprod[((size_t)j * kSubs + u) * 256 + threadIdx.x];
    return P;
}

__device__ __forceinline__ float slice_T_in(const SliceArgs &sl, uint32_t j, uint32_t k) {
    float T = 1.0f;
    for (uint32_t q = 0; q < k; q++) T *= slice_prod(sl, j - k + q);
    return T;
}

// Pass 1: the (1 - a) product of every slice but each tile's last.
template <int TW, int TH>
__global__ __launch_bounds__(256) void k_slice_prod(const gsr_splat *__restrict__ splats,
                                                    const uint32_t *__restrict__ inst,
                                                    const uint32_t *__restrict__ ranges, int W, int H, int ntx,
                                                    int T, SliceArgs sl) {
    __shared__ float4 sA[257], sB[257], sC[257];
    write_null_slot(sA, sB, sC);
    const uint32_t n = min(*sl.count, sl.cap);
    for (uint64_t ju = blockIdx.x; ju < (uint64_t)n * kSubs; ju += gridDim.x) {
        const uint32_t j = (uint32_t)(ju / kSubs), u = (uint32_t)(ju % kSubs);
        const uint2 si = sl.info[j];
        if (si.x == kNoSlice || si.y + 1 == sl.tile_slices[si.x]) continue;
        const TileGeom t = tile_geom<TW, TH>(si.x, T, ntx, W, H);
        const uint32_t start = ranges[2 * si.x], end = ranges[2 * si.x + 1];
        const uint32_t lo = min(start + si.y * kSliceLen + u * kSubLen, end), hi = min(lo + kSubLen, end);
        PixelWalk pw = walk_start(t, 1.0f);
        composite<kKeepTrans>(splats, inst, start, lo, hi, t, sA, sB, sC, pw, nullptr, 0u, 0u);
        sl.tprod[(size_t)ju * 256 + threadIdx.x] = (t.inside && pw.fxl == kGone) ? 0.0f : pw.Tr;
    }
}

// Pass 3: per pixel, the slices' results in order.  Afterwards each slice's colour and depth
// result is replaced by the sum of those behind it (up to the slice in which the pixel
// terminated; zero for slices it never reached), and each slice's transmittance by the one behind
// it (T_final for the terminating slice and those after it): the state from which the backward
// starts a slice.
template <int TW, int TH>
__global__ __launch_bounds__(256) void k_slice_merge(const uint32_t *__restrict__ ranges,
                                                     const gsr_camera *__restrict__ cams, int W, int H, int ntx,
                                                     int T, SliceArgs sl, float *__restrict__ rgb,
                                                     float *__restrict__ depth, float *__restrict__ Tfin,
                                                     uint32_t *__restrict__ last) {
    const uint32_t n = min(*sl.count, sl.cap);
    for (uint32_t j = blockIdx.x; j < n; j += gridDim.x) {
        const uint2 si = sl.info[j];
        if (si.x == kNoSlice || si.y != 0) continue;
        const TileGeom t = tile_geom<TW, TH>(si.x, T, ntx, W, H);
        if (!t.inside) continue;
        const uint32_t K = sl.tile_slices[si.x];
        float Tin = 1.0f, Tr = 1.0f, c0 = 0.f, c1 = 0.f, c2 = 0.f, dd = 0.f;
        uint32_t lst = 0, kt = K - 1;  // kt: the last slice the pixel composited
        for (uint32_t k = 0; k < K; k++) {
            if (Tin < GSR_T_MIN) {  // terminated in an earlier slice
                kt = k - 1;
                break;
            }
            const size_t q = (size_t)(j + k) * 256 + threadIdx.x;
            const float4 pc = sl.part[q];
            const uint2 p2 = sl.part2[q];
            c0 += pc.x;
            c1 += pc.y;
            c2 += pc.z;
            dd += pc.w;
            const float To = __uint_as_float(p2.x);
            Tr = fabsf(To);
            lst = p2.y ? p2.y : lst;
            if (To < 0.0f) {  // terminated in this slice
                kt = k;
                break;
            }
            if (k + 1 < K) Tin *= slice_prod(sl, j + k);
        }
        {
            float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
            for (uint32_t k = K; k-- > 0;) {
                const size_t q = (size_t)(j + k) * 256 + threadIdx.x;
                if (k > kt) {
                    sl.part[q] = acc;
                    sl.part2[q].x = __float_as_uint(Tr);
                    continue;
                }
                const float4 pc = sl.part[q];
                sl.part[q] = acc;
                if (k == kt) sl.part2[q].x = __float_as_uint(Tr);
                acc.x += pc.x;
                acc.y += pc.y;
                acc.z += pc.z;
                acc.w += pc.w;
            }
        }
        const gsr_camera &cam = cams[t.v];
        const int64_t P = (int64_t)W * H;
        const int64_t pix = (int64_t)t.py * W + t.px;
        rgb[(int64_t)t.v * 3 * P + pix] = __builtin_fmaf(Tr, cam.bg[0], c0);
        rgb[(int64_t)t.v * 3 * P + P + pix] = __builtin_fmaf(Tr, cam.bg[1], c1);
        rgb[(int64_t)t.v * 3 * P + 2 * P + pix] = __builtin_fmaf(Tr, cam.bg[2], c2);
        depth[(int64_t)t.v * P + pix] = dd;
        Tfin[(int64_t)t.v * P + pix] = Tr;
        last[(int64_t)t.v * P + pix] = lst;
    }
}

// One 256-lane workgroup per (view, tile) in `order` (longest list first), one pixel per lane.
// With slices (sl.grid > 0) the first sl.grid workgroups composite the slices of the long tiles
// (pass 2), and the long tiles' own workgroups return at once.  COUNT: the contributor counts are
// written to ncon (no slices then).
template <int TW, int TH, bool STORE, bool COUNT = false>
__global__ __launch_bounds__(256) void k_render_fwd(const gsr_splat *__restrict__ splats,
                                                    const uint32_t *__restrict__ inst,
                                                    const uint32_t *__restrict__ ranges,
                                                    const uint32_t *__restrict__ order,
                                                    const gsr_camera *__restrict__ cams, int W, int H, int ntx,
                                                    int T, float *__restrict__ rgb, float *__restrict__ depth,
                                                    float *__restrict__ Tfin, uint32_t *__restrict__ last,
                                                    uint32_t *__restrict__ ncon, const uint32_t *__restrict__ coff,
                                                    uint32_t *__restrict__ clist, uint32_t ccap, SliceArgs sl) {
    static_assert(TW * TH == 256, "one pixel per lane");
    __shared__ float4 sA[257], sB[257], sC[257];
    write_null_slot(sA, sB, sC);
    if (blockIdx.x < sl.grid) {
        const uint32_t n = min(*sl.count, sl.cap);
        for (uint32_t j = blockIdx.x; j < n; j += sl.grid) {
            const uint2 si = sl.info[j];
            if (si.x == kNoSlice) continue;
            const TileGeom t = tile_geom<TW, TH>(si.x, T, ntx, W, H);
            const uint32_t start = ranges[2 * si.x], end = ranges[2 * si.x + 1];
            const uint32_t lo = start + si.y * kSliceLen, hi = min(lo + kSliceLen, end);
            const float Tin = slice_T_in(sl, j, si.y);
            PixelWalk pw = walk_start(t, Tin);
            composite<kKeepImage>(splats, inst, start, lo, hi, t, sA, sB, sC, pw, nullptr, 0u, 0u);
            const bool term = t.inside && Tin >= GSR_T_MIN && pw.fxl == kGone;
            sl.part[(size_t)j * 256 + threadIdx.x] = make_float4(pw.c0, pw.c1, pw.c2, pw.dd);
            sl.part2[(size_t)j * 256 + threadIdx.x] = make_uint2(__float_as_uint(term ? -pw.Tr : pw.Tr), pw.lst);
        }
        return;
    }
    const uint32_t b = blockIdx.x - sl.grid, nb = gridDim.x - sl.grid;
    const uint32_t item = order ? order[b] : xcd_remap(b, nb);
    if (sl.grid && sl.tile_slices[item]) return;  // composited in slices
    const TileGeom t = tile_geom<TW, TH>(item, T, ntx, W, H);
    const uint32_t start = ranges[2 * item], end = ranges[2 * item + 1];
    uint32_t cbase = 0;
    if (STORE && t.inside) cbase = coff[(int64_t)t.v * W * H + (int64_t)t.py * W + t.px];
    PixelWalk pw = walk_start(t, 1.0f);
    constexpr int KEEP = STORE ? kKeepStore : COUNT ? kKeepCount : kKeepImage;
    composite<KEEP>(splats, inst, start, start, end, t, sA, sB, sC, pw, clist, cbase, ccap);
    if (!t.inside || STORE) return;
    const gsr_camera &cam = cams[t.v];
    const int64_t P = (int64_t)W * H;
    const int64_t pix = (int64_t)t.py * W + t.px;
    rgb[(int64_t)t.v * 3 * P + pix] = __builtin_fmaf(pw.Tr, cam.bg[0], pw.c0);
    rgb[(int64_t)t.v * 3 * P + P + pix] = __builtin_fmaf(pw.Tr, cam.bg[1], pw.c1);
    rgb[(int64_t)t.v * 3 * P + 2 * P + pix] = __builtin_fmaf(pw.Tr, cam.bg[2], pw.c2);
    depth[(int64_t)t.v * P + pix] = pw.dd;
    Tfin[(int64_t)t.v * P + pix] = pw.Tr;
    last[(int64_t)t.v * P + pix] = pw.lst;
    if (COUNT) ncon[(int64_t)t.v * P + pix] = pw.nc;
}

// ---- inclusive scans over lane order, in groups of 32 or 16 lanes ----------------------------
// In place, one DPP-sourced VALU op per step: row shifts by 1, 2, 4, 8 scan each 16-lane row,
// then (for groups of 32) the row broadcast of lane 15 carries row 0's total into row 1 and row
// 2's into row 3.  A lane whose source lies outside its row (row_shr without bound_ctrl) or whose
// row is masked off (row_mask) is not written and keeps its value, which is exactly the identity
// step of the scan.  A VALU write of a register needs two wait states before a DPP read of it.
// The whole wave must be active.
// Two independent scans run interleaved: each DPP op's source was written two instructions
// earlier (the other scan's op and an s_nop 0), which covers the same two wait states.  ka and
// kb are values the caller derived from the inputs and needs afterwards: naming them as operands
// makes them ready before the scan, so the scanned registers need no saved copies.
// half_*: groups of 32 lanes (rows 0-1 and rows 2-3: the lane-15 broadcast is the last step);
// row_*: groups of 16 lanes (each row on its own: the row shifts alone).
__device__ __forceinline__ void half_incl_prod2(float &a, float &b, float ka, float kb) {
    asm volatile(
        "s_nop 1\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_mul_f32_dpp %1, %1, %1 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_mul_f32_dpp %1, %1, %1 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_mul_f32_dpp %1, %1, %1 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_mul_f32_dpp %1, %1, %1 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_mul_f32_dpp %1, %1, %1 row_bcast:15 row_mask:0xa bank_mask:0xf"
        : "+v"(a), "+v"(b)
        : "v"(ka), "v"(kb));
}
__device__ __forceinline__ void half_incl_sum2(float &a, float &b, float ka, float kb) {
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_add_f32_dpp %0, %0, %0 row_bcast:15 row_mask:0xa bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_bcast:15 row_mask:0xa bank_mask:0xf"
        : "+v"(a), "+v"(b)
        : "v"(ka), "v"(kb));
}
__device__ __forceinline__ void row_incl_prod2(float &a, float &b, float ka, float kb) {
    asm volatile(
        "s_nop 1\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_mul_f32_dpp %1, %1, %1 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_mul_f32_dpp %1, %1, %1 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_mul_f32_dpp %1, %1, %1 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_mul_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_mul_f32_dpp %1, %1, %1 row_shr:8 row_mask:0xf bank_mask:0xf"
        : "+v"(a), "+v"(b)
        : "v"(ka), "v"(kb));
}
__device__ __forceinline__ void row_incl_sum2(float &a, float &b, float ka, float kb) {
    asm volatile(
        "s_nop 1\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:1 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:2 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:4 row_mask:0xf bank_mask:0xf\n\t"
        "s_nop 0\n\t"
        "v_add_f32_dpp %0, %0, %0 row_shr:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_add_f32_dpp %1, %1, %1 row_shr:8 row_mask:0xf bank_mask:0xf"
        : "+v"(a), "+v"(b)
        : "v"(ka), "v"(kb));
}
template <int GL>
__device__ __forceinline__ void group_incl_prod2(float &a, float &b, float ka, float kb) {
    static_assert(GL == 32 || GL == 16, "lane groups of 32 or 16");
    if constexpr (GL == 32) half_incl_prod2(a, b, ka, kb);
    else row_incl_prod2(a, b, ka, kb);
}
template <int GL>
__device__ __forceinline__ void group_incl_sum2(float &a, float &b, float ka, float kb) {
    static_assert(GL == 32 || GL == 16, "lane groups of 32 or 16");
    if constexpr (GL == 32) half_incl_sum2(a, b, ka, kb);
    else row_incl_sum2(a, b, ka, kb);
}

// Shared memory of the backward of one tile (the staged splats keep the forward's null slot 256).
struct BwdLds {
    float4 sA[257], sB[257], sC[257];
    float sAcc[10][256];
    uint8_t sList[4][256];
    float4 sPG[4][64];    // dL/dC (3), dL/dD
    float2 sPS[4][64];    // transmittance and suffix sum behind the chunks done so far
    uint32_t sPL[4][64];  // last composited position of each pixel
    uint32_t s_max;
};

// The calling lane's pixel state for the backward: final transmittance, last composited position
// (0 for a pixel outside the image) and upstream gradients dL/dC, dL/dD.
struct PixelGrad {
    float Tr, G0, G1, G2, GD;
    uint32_t last;
};

// The suffix behind a whole tile: the background term T_final (dL/dC . bg).
__device__ __forceinline__ float bg_suffix(const PixelGrad &pg, const gsr_camera &cam) {
    return pg.Tr * (pg.G0 * cam.bg[0] + pg.G1 * cam.bg[1] + pg.G2 * cam.bg[2]);
}

// Backward of one (view, tile) work item, Gaussian-major.  The tile's instances up to the deepest
// pixel's last contributor are staged back to front in batches of 256.  Each wave compacts the
// batch to the Gaussians that reach its pixel sub-rectangle and cuts them, deepest first, into
// chunks of 32 (the last one of 16 when at most 16 remain): lane l holds the (l % 32)-th deepest,
// and the two halves of the wave (four quarters for a chunk of 16) work on different pixels of
// the same Gaussians.  For each of its pixels every lane evaluates its Gaussian; an inclusive
// product scan of 1 / (1 - a) over the lane group recovers the transmittance in front of each
// Gaussian from the pixel's transmittance behind the chunk, and an inclusive sum scan of
// w (dL/dC . c + dL/dD z) gives what lies behind it.  Pixel state (upstream gradient,
// transmittance and suffix behind the chunks done so far) sits in LDS and is read by broadcast.
// Per lane, the mean and conic gradients accumulate as
// the five moments sum dP (dx, dy, dx^2, dx dy, dy^2) of the exponent gradient dP, mapped through
// the Cholesky factor once per chunk.  Gradients then accumulate in LDS across waves (ds_add_f32
// per staged slot) and leave as one plain 40-byte record per instance, stored at the instance's
// emission index: the records of one (view, Gaussian) pair are contiguous there, and the
// projection backward sums them in a fixed order, so no global atomics are needed.  The four
// waves' adds to one slot come in a run-dependent order, so gradients repeat from run to run only
// up to float rounding.  Block-uniform arguments except the pixel state pg and S0.
// [lo, hi) (positions in the tile's list) is the part of the tile this call handles: the whole tile,
// or one depth slice of a long tile.  pg.Tr is the pixel's transmittance behind that part and S0
// the suffix behind it: T_final (dL/dC . bg) for the whole tile, plus dL/dC . C_behind + dL/dD
// D_behind (the colour and depth composited behind the slice) for a slice.
template <int TW, int TH>
__device__ __forceinline__ void tile_backward(const gsr_splat *__restrict__ splats, const uint32_t *__restrict__ inst,
                                              const uint32_t *__restrict__ inst_emit, uint32_t item, uint32_t start,
                                              uint32_t lo, uint32_t hi, int ntx, int T, const gsr_camera &cam,
                                              const PixelGrad &pg, float S0, BwdLds &L, float *__restrict__ dinst) {
    float4 *const sA = L.sA, *const sB = L.sB, *const sC = L.sC;
    auto &sAcc = L.sAcc;
    auto &sList = L.sList;
    auto &sPG = L.sPG;
    auto &sPS = L.sPS;
    auto &sPL = L.sPL;
    uint32_t &s_max = L.s_max;
    const int tile = item % T;
    const int tx = tile % ntx, ty = tile / ntx;
    const int bx = (tx * TW) & ~31, by = (ty * TH) & ~31;
    const double ox = (double)bx, oy = (double)by;
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    float wx0, wx1, wy0, wy1;
    wave_box<TW>(tx * TW - bx, ty * TH - by, w, wx0, wx1, wy0, wy1);
    // centre of the wave's first pixel (the wave's 64 pixels are TW-wide rows)
    static_assert(TW % 8 == 0, "packed chunks assume 8 | TW");
    const float fxw = (float)(tx * TW - bx) + 0.5f, fyw = (float)(ty * TH - by + w * (64 / TW)) + 0.5f;
    const uint32_t mylast = pg.last;
    {
        sPG[w][lane] = make_float4(pg.G0, pg.G1, pg.G2, pg.GD);
        sPS[w][lane] = make_float2(pg.Tr, S0);
        sPL[w][lane] = mylast;
        if (threadIdx.x == 0) s_max = 0;
    }
    for (int q = threadIdx.x; q < 2560; q += 256) (&sAcc[0][0])[q] = 0.f;
    __syncthreads();
    if (mylast) atomicMax(&s_max, mylast);
    // the deepest last contributor of this wave's pixels
    uint32_t wmax = mylast;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wmax = max(wmax, (uint32_t)__shfl_xor((int)wmax, off));
    __syncthreads();
    const uint32_t nl = min(s_max, hi);
    // instances behind every pixel's last contributor receive a zero record
    for (uint32_t k = start + max(nl, lo) + threadIdx.x; k < start + hi; k += 256) {
        float2 *rec = reinterpret_cast<float2 *>(dinst + (int64_t)inst_emit[k] * GSR_SPLAT_GRAD_FLOATS);
#pragma unroll
        for (int e = 0; e < 5; e++) rec[e] = make_float2(0.f, 0.f);
    }
    const float kap = (float)GSR_KAPPA;
    const float nln2 = -(float)GSR_LN2;
    for (int bend = (int)nl; bend > (int)lo; bend -= 256) {
        const int b0 = bend - 256 > (int)lo ? bend - 256 : (int)lo;
        const int cnt = bend - b0;
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const uint32_t gid = inst[start + b0 + threadIdx.x];
            float4 A, B, C;
            stage_splat(splats, gid, ox, oy, A, B, C);
            sA[threadIdx.x] = A;
            sB[threadIdx.x] = B;
            sC[threadIdx.x] = C;
        }
        __syncthreads();
        // compact the staged Gaussians that reach this wave's pixels, deepest first
        int nw = 0;
        for (int g = 3; g >= 0; g--) {
            const int slot = g * 64 + lane;
            bool r = false;
            if (slot < cnt && (uint32_t)(b0 + slot) < wmax)
                r = ellipse_meets_box(sA[slot], sB[slot], wx0, wx1, wy0, wy1);
            const uint64_t m = __ballot(r);
            if (r) {
                const uint64_t above = lane == 63 ? 0ull : (m >> (lane + 1));
                sList[w][nw + __popcll(above)] = (uint8_t)slot;
            }
            nw += __popcll(m);
        }
        __builtin_amdgcn_wave_barrier();  // the wave reads back what its lanes just wrote
        // One chunk of the compacted list, c0 onwards: lane l holds the chunk's (l % GL)-th
        // deepest Gaussian for pixel group l / GL.  The 2 (GL = 32) or 4 (GL = 16) groups of
        // lanes work on different pixels of the same Gaussians at once, and their sums meet
        // before the LDS adds.  Chunks of 32 rather than one of 64 across the wave: the last,
        // partial chunk of a wave's list leaves fewer lanes empty, and a 32-lane scan is one
        // DPP step shorter.
        auto chunk = [&](auto glc, int c0) {
            constexpr int GL = decltype(glc)::value;
            constexpr int NG = 64 / GL;
            const int gl = lane % GL, grp = lane / GL;
            const int rem = nw - c0;
            const bool gvalid = gl < rem;
            const int slot = gvalid ? sList[w][c0 + gl] : 0;
            const float4 A = gvalid ? sA[slot] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 B = gvalid ? sB[slot] : make_float4(0.f, -1.f, 0.f, 0.f);
            const float4 C = gvalid ? sC[slot] : make_float4(0.f, 0.f, 0.f, 0.f);
            const uint32_t pos = (uint32_t)(b0 + slot);
            const uint32_t posv = gvalid ? pos : 0xffffffffu;  // never below a last contributor
            // frontmost position of the chunk: the last valid lane of the first group
            const int lastlane = (rem < GL ? rem : GL) - 1;
            const uint32_t cfront = (uint32_t)__builtin_amdgcn_readlane((int)pos, lastlane);
            float cr = 0.f, cg = 0.f, cb = 0.f, cd = 0.f, go = 0.f;
            float mx = 0.f, my = 0.f, mxx = 0.f, mxy = 0.f, myy = 0.f;
            const float kz = nln2 * B.z;
            // One iteration: this group's pixels q0 and q1 of one row, their offsets dx0, dx1 from
            // the mean and the row's dy terms.  Returns false when no Gaussian of the chunk reaches
            // either pixel; else g0, g1 = 2^-P dL/da of the lane's Gaussian at the two pixels (zero
            // where it does not blend or the clamp holds alpha), with the colour and depth sums and
            // the pixels' state updated.
            auto pixel_pair = [&](int q0, int q1, float dx0, float dx1, float l21dy, float u22, float &g0,
                                  float &g1) -> bool {
                const uint32_t l0 = sPL[w][q0], l1 = sPL[w][q1];
                if (__ballot(cfront < l0 || cfront < l1) == 0) return false;
                const float4 pg0 = sPG[w][q0], pg1 = sPG[w][q1];
                const float2 s0 = sPS[w][q0], s1 = sPS[w][q1];
                const float T0 = s0.x, S0 = s0.y, T1 = s1.x, S1 = s1.y;
                // Each operation is the one blend_exponent performs: the exponents, and so every
                // contribute / skip decision, are bit-identical to the forward's.
                const float u10 = __builtin_fmaf(A.z, dx0, l21dy), u11 = __builtin_fmaf(A.z, dx1, l21dy);
                const float P0 = __builtin_fmaf(u10, u10, u22), P1 = __builtin_fmaf(u11, u11, u22);
                const bool act0 = posv < l0 && P0 <= B.y;
                const bool act1 = posv < l1 && P1 <= B.y;
                if (__ballot(act0 || act1) == 0) return false;  // no Gaussian of the chunk reaches them
                const float e0 = act0 ? __builtin_amdgcn_exp2f(-P0) : 0.f;
                const float e1 = act1 ? __builtin_amdgcn_exp2f(-P1) : 0.f;
                const float ar0 = B.z * e0, ar1 = B.z * e1;
                const float a0 = fminf(ar0, GSR_ALPHA_MAX), a1 = fminf(ar1, GSR_ALPHA_MAX);
                const float om0 = 1.0f - a0, om1 = 1.0f - a1;
                // the scans overwrite their operands in place, so they run on copies of what is
                // needed afterwards: here the product of 1 / (1 - a) over the chunk's Gaussians
                // up to each one (deepest first), which spares dividing by the product of (1 - a)
                const float rom0 = __builtin_amdgcn_rcpf(om0), rom1 = __builtin_amdgcn_rcpf(om1);
                float R0 = rom0, R1 = rom1;
                group_incl_prod2<GL>(R0, R1, rom0, rom1);
                // transmittance in front of each Gaussian: T behind the chunk times that product
                // (at most 1e4, since T behind is at least T_final >= 1e-4)
                const float Tb0 = T0 * R0;
                const float Tb1 = T1 * R1;
                const float w0 = a0 * Tb0, w1 = a1 * Tb1;
                const float gs0 =
                    __builtin_fmaf(pg0.x, C.x, __builtin_fmaf(pg0.y, C.y, __builtin_fmaf(pg0.z, C.z, pg0.w * B.w)));
                const float gs1 =
                    __builtin_fmaf(pg1.x, C.x, __builtin_fmaf(pg1.y, C.y, __builtin_fmaf(pg1.z, C.z, pg1.w * B.w)));
                float in0 = w0 * gs0, in1 = w1 * gs1;
                const float sb0 = S0 - in0, sb1 = S1 - in1;
                group_incl_sum2<GL>(in0, in1, sb0, sb1);
                // everything behind each Gaussian
                const float Sa0 = sb0 + in0, Sa1 = sb1 + in1;
                const float d0 = __builtin_fmaf(Tb0, gs0, -Sa0 * rom0);
                const float d1 = __builtin_fmaf(Tb1, gs1, -Sa1 * rom1);
                // colour and depth: weight w = a T (zero for lanes that do not blend)
                cr = __builtin_fmaf(pg0.x, w0, __builtin_fmaf(pg1.x, w1, cr));
                cg = __builtin_fmaf(pg0.y, w0, __builtin_fmaf(pg1.y, w1, cg));
                cb = __builtin_fmaf(pg0.z, w0, __builtin_fmaf(pg1.z, w1, cb));
                cd = __builtin_fmaf(pg0.w, w0, __builtin_fmaf(pg1.w, w1, cd));
                // unclamped alpha = o 2^-P: dL/do = 2^-P dL/da, dL/dP = -ln2 o (2^-P dL/da)
                // (zero where the clamp holds alpha)
                const bool lin0 = act0 && ar0 <= GSR_ALPHA_MAX, lin1 = act1 && ar1 <= GSR_ALPHA_MAX;
                g0 = (lin0 ? e0 : 0.f) * d0;
                g1 = (lin1 ? e1 : 0.f) * d1;
                // the pixels' state in front of this chunk, kept by each group's frontmost lane
                // (inactive lanes carry a = 0)
                if (gl == GL - 1) {
                    sPS[w][q0] = make_float2(Tb0, S0 + in0);
                    sPS[w][q1] = make_float2(Tb1, S1 + in1);
                }
                return true;
            };
            // The wave's pixels lie row-major in a TW-wide box.  Each iteration takes two pixels
            // per group, NG apart in one row: group grp covers the columns grp + NG k of every
            // row.  Their chains are independent, which keeps the SIMD busy through the scan and
            // transcendental latencies.
            if constexpr (TW / NG <= 4) {
                // Few columns per lane: their offsets dx from the mean are formed once per chunk,
                // the dy terms once per row, and the exponent-gradient moments accumulate per
                // column (sum of g) and per row (sums of g and g dx), with kappa_z = -ln2 o
                // applied once at the end.
                constexpr int HPR = TW / (2 * NG), NCOL = 2 * HPR;
                float dxc[NCOL], Gc[NCOL];
                const float fxg = fxw + (float)grp;  // exact: pixel centres are small half-integers
#pragma unroll
                for (int k = 0; k < NCOL; k++) {
                    dxc[k] = (fxg + (float)(NG * k)) - A.x;
                    Gc[k] = 0.f;
                }
                float fyr = fyw;
                for (int r = 0; r < 64 / TW; r++, fyr += 1.0f) {
                    const float dy = fyr - A.y;
                    const float l21dy = A.w * dy, u2 = B.x * dy, u22 = u2 * u2;
                    float rs = 0.f, rx = 0.f;
#pragma unroll
                    for (int h = 0; h < HPR; h++) {
                        const int q0 = r * TW + 2 * NG * h + grp;
                        float g0, g1;
                        if (!pixel_pair(q0, q0 + NG, dxc[2 * h], dxc[2 * h + 1], l21dy, u22, g0, g1)) continue;
                        Gc[2 * h] += g0;
                        Gc[2 * h + 1] += g1;
                        rs += g0 + g1;
                        rx = __builtin_fmaf(g0, dxc[2 * h], __builtin_fmaf(g1, dxc[2 * h + 1], rx));
                    }
                    my = __builtin_fmaf(rs, dy, my);
                    myy = __builtin_fmaf(rs * dy, dy, myy);
                    mxy = __builtin_fmaf(rx, dy, mxy);
                }
#pragma unroll
                for (int k = 0; k < NCOL; k++) {
                    go += Gc[k];
                    const float t = Gc[k] * dxc[k];
                    mx += t;
                    mxx = __builtin_fmaf(t, dxc[k], mxx);
                }
                mx *= kz;
                my *= kz;
                mxx *= kz;
                mxy *= kz;
                myy *= kz;
            } else {
                for (int p = 0; p < 64; p += 2 * NG) {
                    // this group's two pixels: 2 NG divides TW, so q0 and q1 sit in the row of p,
                    // at columns p % TW + grp and + NG
                    const int q0 = p + grp, q1 = p + NG + grp;
                    const float fxp = fxw + (float)(p % TW);
                    const float fx0 = fxp + (float)grp, fx1 = fxp + (float)(NG + grp);
                    const float fy0 = fyw + (float)(p / TW);
                    // the two pixels share a row, so dy and the terms of the exponent that depend
                    // on dy alone are formed once
                    const float dy = fy0 - A.y;
                    const float l21dy = A.w * dy, u2 = B.x * dy, u22 = u2 * u2;
                    const float dx0 = fx0 - A.x, dx1 = fx1 - A.x;
                    float g0, g1;
                    if (!pixel_pair(q0, q1, dx0, dx1, l21dy, u22, g0, g1)) continue;
                    go += g0 + g1;
                    const float dP0 = kz * g0, dP1 = kz * g1;
                    mx = __builtin_fmaf(dP0, dx0, __builtin_fmaf(dP1, dx1, mx));
                    const float sP = dP0 + dP1;
                    my = __builtin_fmaf(sP, dy, my);
                    const float qq0 = dP0 * dx0, qq1 = dP1 * dx1;
                    mxx = __builtin_fmaf(qq0, dx0, __builtin_fmaf(qq1, dx1, mxx));
                    mxy = __builtin_fmaf(qq0 + qq1, dy, mxy);
                    myy = __builtin_fmaf(sP * dy, dy, myy);
                }
            }
            {
                // the groups' sums for one Gaussian meet in the first group
                float *const sums[10] = {&cr, &cg, &cb, &cd, &go, &mx, &my, &mxx, &mxy, &myy};
#pragma unroll
                for (int e = 0; e < 10; e++) {
                    float x = *sums[e];
#pragma unroll
                    for (int off = GL; off < 64; off <<= 1) x += __shfl_xor(x, off);
                    *sums[e] = x;
                }
            }
            if (gvalid && grp == 0) {
                // P = |L^T D|^2 with D = pixel - mean: dP/dmean = -2 L L^T D, dP/dQ = kappa D D^T
                const float l11 = A.z, l21 = A.w, l22 = B.x;
                const float m1 = __builtin_fmaf(l11, mx, l21 * my);
                float acc[10];
                acc[0] = -2.0f * (l11 * m1);
                acc[1] = -2.0f * __builtin_fmaf(l21, m1, l22 * l22 * my);
                acc[2] = kap * mxx;
                acc[3] = 2.0f * kap * mxy;
                acc[4] = kap * myy;
                acc[5] = go;
                acc[6] = cr;
                acc[7] = cg;
                acc[8] = cb;
                acc[9] = cd;
#pragma unroll
                for (int e = 0; e < 10; e++)
                    if (acc[e] != 0.f) atomicAdd(&sAcc[e][slot], acc[e]);
            }
        };
        for (int c0 = 0; c0 < nw;) {
            if (nw - c0 > 16) {
                chunk(std::integral_constant<int, 32>{}, c0);
                c0 += 32;
            } else {
                chunk(std::integral_constant<int, 16>{}, c0);
                c0 += 16;
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            float2 *rec = reinterpret_cast<float2 *>(
                dinst + (int64_t)inst_emit[start + b0 + threadIdx.x] * GSR_SPLAT_GRAD_FLOATS);
#pragma unroll
            for (int e = 0; e < 5; e++) {
                rec[e] = make_float2(sAcc[2 * e][threadIdx.x], sAcc[2 * e + 1][threadIdx.x]);
                sAcc[2 * e][threadIdx.x] = 0.f;
                sAcc[2 * e + 1][threadIdx.x] = 0.f;
            }
        }
    }
}

// The depth slices of the long tiles, for the first sl.grid workgroups of a backward launch: each
// slice's backward from the state behind it that the sliced forward's merge left in the slice
// results (transmittance behind the slice; colour and depth composited behind it).
// grad(t, pix, pg) fills the pixel's upstream gradient pg.G0..GD.
template <int TW, int TH, class Grad>
__device__ __forceinline__ void slices_backward(const gsr_splat *__restrict__ splats, const uint32_t *__restrict__ inst,
                                                const uint32_t *__restrict__ inst_emit,
                                                const uint32_t *__restrict__ ranges,
                                                const gsr_camera *__restrict__ cams, int W, int H, int ntx, int T,
                                                const float *__restrict__ Tfin, const uint32_t *__restrict__ last,
                                                const SliceArgs &sl, BwdLds &L, float *__restrict__ dinst, Grad grad) {
    const int64_t P = (int64_t)W * H;
    const uint32_t n = min(*sl.count, sl.cap);
    for (uint32_t j = blockIdx.x; j < n; j += sl.grid) {
        const uint2 si = sl.info[j];
        if (si.x == kNoSlice) continue;
        __syncthreads();  // every lane has left the previous slice's shared state
        const TileGeom t = tile_geom<TW, TH>(si.x, T, ntx, W, H);
        const int64_t pix = (int64_t)t.py * W + t.px;
        const gsr_camera &cam = cams[t.v];
        const uint32_t start = ranges[2 * si.x], len = ranges[2 * si.x + 1] - start;
        const uint32_t lo = si.y * kSliceLen, hi = min(lo + kSliceLen, len);
        PixelGrad pg{1.f, 0.f, 0.f, 0.f, 0.f, 0u};
        float S0 = 0.f;
        if (t.inside) {
            grad(t, pix, pg);
            pg.last = last[(int64_t)t.v * P + pix];
            const size_t q = (size_t)j * 256 + threadIdx.x;
            const float4 cb = sl.part[q];  // colour and depth behind the slice
            PixelGrad fin = pg;
            fin.Tr = Tfin[(int64_t)t.v * P + pix];
            S0 = bg_suffix(fin, cam) + (pg.G0 * cb.x + pg.G1 * cb.y + pg.G2 * cb.z + pg.GD * cb.w);
            pg.Tr = fabsf(__uint_as_float(sl.part2[q].x));  // transmittance behind the slice
        }
        tile_backward<TW, TH>(splats, inst, inst_emit, si.x, start, lo, hi, ntx, T, cam, pg, S0, L, dinst);
    }
}

template <int TW, int TH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_render_bwd(
    const gsr_splat *__restrict__ splats, const uint32_t *__restrict__ inst, const uint32_t *__restrict__ inst_emit,
    const uint32_t *__restrict__ ranges, const uint32_t *__restrict__ order, const gsr_camera *__restrict__ cams, int W,
    int H, int ntx, int T, const float *__restrict__ Tfin, const uint32_t *__restrict__ last,
    const float *__restrict__ dLdrgb, const float *__restrict__ dLddepth, float *__restrict__ dinst, SliceArgs sl) {
    __shared__ BwdLds L;
    const int64_t P = (int64_t)W * H;
    auto grad = [&](const TileGeom &t, int64_t pix, PixelGrad &pg) {
        pg.G0 = dLdrgb[(int64_t)t.v * 3 * P + pix];
        pg.G1 = dLdrgb[(int64_t)t.v * 3 * P + P + pix];
        pg.G2 = dLdrgb[(int64_t)t.v * 3 * P + 2 * P + pix];
        if (dLddepth) pg.GD = dLddepth[(int64_t)t.v * P + pix];
    };
    if (blockIdx.x < sl.grid) {
        slices_backward<TW, TH>(splats, inst, inst_emit, ranges, cams, W, H, ntx, T, Tfin, last, sl, L, dinst, grad);
        return;
    }
    const uint32_t bk = blockIdx.x - sl.grid, nb = gridDim.x - sl.grid;
    const uint32_t item = order ? order[bk] : xcd_remap(bk, nb);
    if (sl.grid && sl.tile_slices[item]) return;  // its backward runs in depth slices
    const TileGeom t = tile_geom<TW, TH>(item, T, ntx, W, H);
    const int64_t pix = (int64_t)t.py * W + t.px;
    PixelGrad pg{1.f, 0.f, 0.f, 0.f, 0.f, 0u};
    if (t.inside) {
        pg.Tr = Tfin[(int64_t)t.v * P + pix];
        pg.last = last[(int64_t)t.v * P + pix];
        grad(t, pix, pg);
    }
    const uint32_t start = ranges[2 * item];
    tile_backward<TW, TH>(splats, inst, inst_emit, item, start, 0u, ranges[2 * item + 1] - start, ntx, T, cams[t.v], pg,
                          bg_suffix(pg, cams[t.v]), L, dinst);
}

// ---- fused persistent step: forward, L1 loss gradient and backward of each tile ----------------
// Eq. 9-10 with the all-ones mask and lambda_ssim = 0 is a per-pixel loss, so one workgroup can
// composite a tile, form its pixels' loss gradient in registers and run the tile's backward at
// once: the images and the loss gradient never make a round trip through memory for the
// backward.  Work items come from a device queue: first the depth slices of the long tiles, then
// the view-tiles in longest-first order.  A long tile is finished by the workgroup that completes
// its last slice (the completion counter tells it which): it merges the slices, forms the loss
// gradient and runs the tile's backward, so no workgroup ever waits for another.
struct StepArgs {
    const float *trgb, *tdepth;  // targets [S][3][H][W], [S][H][W] (tdepth may be null)
    const int32_t *tidx;         // [V] target slot of each view (null: slot v)
    float lam;                   // depth weight lambda_d
    double *item_loss;           // [V*T] sum over the view-tile's pixels of their loss terms
    uint32_t *queue;             // [1] next work item, 0 before the launch
    uint32_t *slices_done;       // [V*T] finished slices of each long tile, 0 before the launch
};

// L1 loss term of one pixel (colour channels summed, plus lambda_d times the depth term) and its
// gradient: dL/dC = sign(C - C~) / P, dL/dD = lambda_d sign(D - D~) / P, sign(0) = 0.
__device__ __forceinline__ float l1_pixel(const StepArgs &a, int v, int64_t P, int64_t pix, float r, float g, float b,
                                          float d, PixelGrad &pg) {
    const int64_t slot = a.tidx ? (int64_t)a.tidx[v] : (int64_t)v;
    const float invP = 1.0f / (float)P;
    const float c[3] = {r, g, b};
    float gr[3];
    float l = 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
        const float dl = c[ch] - a.trgb[slot * 3 * P + ch * P + pix];
        l += fabsf(dl);
        gr[ch] = dl > 0.f ? invP : (dl < 0.f ? -invP : 0.f);
    }
    pg.G0 = gr[0];
    pg.G1 = gr[1];
    pg.G2 = gr[2];
    pg.GD = 0.f;
    if (a.tdepth) {
        const float dl = d - a.tdepth[slot * P + pix];
        l += a.lam * fabsf(dl);
        pg.GD = a.lam * (dl > 0.f ? invP : (dl < 0.f ? -invP : 0.f));
    }
    return l;
}

// Writes the pixel's outputs, forms its loss gradient, and stores the view-tile's loss sum.
__device__ __forceinline__ void finish_pixels(const TileGeom &t, uint32_t item, const gsr_camera &cam, int W, int H,
                                              float Tr, float c0, float c1, float c2, float dd, uint32_t lst,
                                              float *__restrict__ rgb, float *__restrict__ depth,
                                              float *__restrict__ Tfin, uint32_t *__restrict__ last,
                                              const StepArgs &a, PixelGrad &pg, double *s_red) {
    const int64_t P = (int64_t)W * H;
    const int64_t pix = (int64_t)t.py * W + t.px;
    pg = PixelGrad{1.f, 0.f, 0.f, 0.f, 0.f, 0u};
    double l = 0.0;
    if (t.inside) {
        const float r = __builtin_fmaf(Tr, cam.bg[0], c0);
        const float g = __builtin_fmaf(Tr, cam.bg[1], c1);
        const float b = __builtin_fmaf(Tr, cam.bg[2], c2);
        rgb[(int64_t)t.v * 3 * P + pix] = r;
        rgb[(int64_t)t.v * 3 * P + P + pix] = g;
        rgb[(int64_t)t.v * 3 * P + 2 * P + pix] = b;
        depth[(int64_t)t.v * P + pix] = dd;
        Tfin[(int64_t)t.v * P + pix] = Tr;
        last[(int64_t)t.v * P + pix] = lst;
        l = (double)l1_pixel(a, t.v, P, pix, r, g, b, dd, pg);
        pg.Tr = Tr;
        pg.last = lst;
    }
    l = wave_sum_d(l);
    if (__lane_id() == 0) s_red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) a.item_loss[item] = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
}

template <int TW, int TH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_render_step(
    const gsr_splat *__restrict__ splats, const uint32_t *__restrict__ inst, const uint32_t *__restrict__ inst_emit,
    const uint32_t *__restrict__ ranges, const uint32_t *__restrict__ order, const gsr_camera *__restrict__ cams,
    int W, int H, int ntx, int T, uint32_t VT, float *__restrict__ rgb, float *__restrict__ depth,
    float *__restrict__ Tfin, uint32_t *__restrict__ last, float *__restrict__ dinst, SliceArgs sl, StepArgs a) {
    __shared__ BwdLds L;
    __shared__ uint32_t s_item, s_flag;
    __shared__ double s_red[4];
    write_null_slot(L.sA, L.sB, L.sC);
    const uint32_t n_sl = sl.grid ? min(*sl.count, sl.cap) : 0u;
    const uint32_t total = n_sl + VT;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t it = s_item;
        __syncthreads();  // every lane has read the item before thread 0 fetches the next one
        if (it >= total) break;
        PixelGrad pg;
        uint32_t item, start, end;
        TileGeom t;
        if (it < n_sl) {
            // one depth slice of a long tile, composited from the transmittance in front of it
            const uint2 si = sl.info[it];
            if (si.x == kNoSlice) continue;
            item = si.x;
            t = tile_geom<TW, TH>(item, T, ntx, W, H);
            start = ranges[2 * item];
            end = ranges[2 * item + 1];
            const uint32_t lo = start + si.y * kSliceLen, hi = min(lo + kSliceLen, end);
            const float Tin = slice_T_in(sl, it, si.y);
            PixelWalk pw = walk_start(t, Tin);
            composite<kKeepImage>(splats, inst, start, lo, hi, t, L.sA, L.sB, L.sC, pw, nullptr, 0u, 0u);
            const bool term = t.inside && Tin >= GSR_T_MIN && pw.fxl == kGone;
            sl.part[(size_t)it * 256 + threadIdx.x] = make_float4(pw.c0, pw.c1, pw.c2, pw.dd);
            sl.part2[(size_t)it * 256 + threadIdx.x] = make_uint2(__float_as_uint(term ? -pw.Tr : pw.Tr), pw.lst);
            // release the slice's results, then count it; the workgroup that completes the tile's
            // last slice acquires every slice's results and finishes the tile
            __threadfence();
            __syncthreads();
            if (threadIdx.x == 0) {
                const uint32_t K = sl.tile_slices[item];
                s_flag = atomicAdd(&a.slices_done[item], 1u) + 1u == K ? 1u : 0u;
                __threadfence();
            }
            __syncthreads();
            if (!s_flag) continue;
            __threadfence();
            const uint32_t j0 = it - si.y, K = sl.tile_slices[item];
            float Tin2 = 1.0f, Tr = 1.0f, c0 = 0.f, c1 = 0.f, c2 = 0.f, dd = 0.f;
            uint32_t lst = 0;
            if (t.inside) {
                for (uint32_t k = 0; k < K; k++) {
                    if (Tin2 < GSR_T_MIN) break;  // terminated in an earlier slice
                    const size_t q = (size_t)(j0 + k) * 256 + threadIdx.x;
                    const float4 pc = sl.part[q];
                    const uint2 p2 = sl.part2[q];
                    c0 += pc.x;
                    c1 += pc.y;
                    c2 += pc.z;
                    dd += pc.w;
                    const float To = __uint_as_float(p2.x);
                    Tr = fabsf(To);
                    lst = p2.y ? p2.y : lst;
                    if (To < 0.0f) break;  // terminated in this slice
                    if (k + 1 < K) Tin2 *= slice_prod(sl, j0 + k);
                }
            }
            finish_pixels(t, item, cams[t.v], W, H, Tr, c0, c1, c2, dd, lst, rgb, depth, Tfin, last, a, pg, s_red);
        } else {
            item = order ? order[it - n_sl] : it - n_sl;
            if (sl.grid && sl.tile_slices[item]) continue;  // composited in slices
            t = tile_geom<TW, TH>(item, T, ntx, W, H);
            start = ranges[2 * item];
            end = ranges[2 * item + 1];
            PixelWalk pw = walk_start(t, 1.0f);
            composite<kKeepImage>(splats, inst, start, start, end, t, L.sA, L.sB, L.sC, pw, nullptr, 0u, 0u);
            finish_pixels(t, item, cams[t.v], W, H, pw.Tr, pw.c0, pw.c1, pw.c2, pw.dd, pw.lst, rgb, depth, Tfin, last,
                          a, pg, s_red);
        }
        tile_backward<TW, TH>(splats, inst, inst_emit, item, start, 0u, end - start, ntx, T, cams[t.v], pg,
                              bg_suffix(pg, cams[t.v]), L, dinst);
        __syncthreads();  // the backward's last flush reads LDS the next item overwrites
    }
}

// Loss of the step: the view-tiles' sums in a fixed order, divided by the pixels per view, added
// to *loss.
__global__ __launch_bounds__(1024) void k_step_loss(const double *__restrict__ item_loss, uint32_t VT, double invP,
                                                    double *__restrict__ loss) {
    __shared__ double s_w[16];
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < VT; i += 1024) acc += item_loss[i];
    acc = wave_sum_d(acc);
    if (__lane_id() == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < 16; k++) s += s_w[k];
        *loss += s * invP;
    }
}

// The render backward of the per-pixel L1 loss (Eq. 9-10, all-ones mask, lambda_ssim = 0): each
// lane forms its pixel's loss term and gradient from the forward's image and the targets (so no
// gradient image is written or read), the workgroup stores its view-tile's loss sum, then runs the
// tile's backward.  One workgroup per view-tile, longest first.
template <int TW, int TH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_render_bwd_l1(
    const gsr_splat *__restrict__ splats, const uint32_t *__restrict__ inst, const uint32_t *__restrict__ inst_emit,
    const uint32_t *__restrict__ ranges, const uint32_t *__restrict__ order, const gsr_camera *__restrict__ cams, int W,
    int H, int ntx, int T, const float *__restrict__ rgb, const float *__restrict__ depth,
    const float *__restrict__ Tfin, const uint32_t *__restrict__ last, float *__restrict__ dinst, StepArgs a,
    SliceArgs sl) {
    __shared__ BwdLds L;
    __shared__ double s_red[4];
    const int64_t P = (int64_t)W * H;
    if (blockIdx.x < sl.grid) {
        slices_backward<TW, TH>(splats, inst, inst_emit, ranges, cams, W, H, ntx, T, Tfin, last, sl, L, dinst,
                                [&](const TileGeom &t, int64_t pix, PixelGrad &pg) {
                                    const int64_t b = (int64_t)t.v * 3 * P + pix;
                                    l1_pixel(a, t.v, P, pix, rgb[b], rgb[b + P], rgb[b + 2 * P],
                                             depth[(int64_t)t.v * P + pix], pg);
                                });
        return;
    }
    const uint32_t bk = blockIdx.x - sl.grid, nb = gridDim.x - sl.grid;
    const uint32_t item = order ? order[bk] : xcd_remap(bk, nb);
    const TileGeom t = tile_geom<TW, TH>(item, T, ntx, W, H);
    const int64_t pix = (int64_t)t.py * W + t.px;
    PixelGrad pg{1.f, 0.f, 0.f, 0.f, 0.f, 0u};
    double l = 0.0;
    if (t.inside) {
        const int64_t b = (int64_t)t.v * 3 * P + pix;
        l = (double)l1_pixel(a, t.v, P, pix, rgb[b], rgb[b + P], rgb[b + 2 * P], depth[(int64_t)t.v * P + pix], pg);
        pg.Tr = Tfin[(int64_t)t.v * P + pix];
        pg.last = last[(int64_t)t.v * P + pix];
    }
    l = wave_sum_d(l);
    if (__lane_id() == 0) s_red[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) a.item_loss[item] = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
    if (sl.grid && sl.tile_slices[item]) return;  // its backward runs in depth slices
    const uint32_t start = ranges[2 * item];
    tile_backward<TW, TH>(splats, inst, inst_emit, item, start, 0u, ranges[2 * item + 1] - start, ntx, T, cams[t.v], pg,
                          bg_suffix(pg, cams[t.v]), L, dinst);
}

// Backward of the stored-contributor mode, pixel-major: every lane walks its own pixel's list of
// composited tile positions back to front (no re-evaluation of Gaussians that did not blend),
// recovering the transmittance in front of each contributor by division.  The tile's instances
// are staged back to front in batches of 256 as in the recompute backward; per batch each lane
// handles the entries of its list that fall inside the batch, and the ten gradient components
// meet in LDS (ds_add_f32 per staged slot) before leaving as one record per instance.
template <int TW, int TH>
__global__ __launch_bounds__(256) void k_render_bwd_stored(const gsr_splat *__restrict__ splats,
                                                           const uint32_t *__restrict__ inst,
                                                           const uint32_t *__restrict__ inst_emit,
                                                           const uint32_t *__restrict__ ranges,
                                                           const uint32_t *__restrict__ order,
                                                           const gsr_camera *__restrict__ cams, int W, int H,
                                                           int ntx, int T, const float *__restrict__ Tfin,
                                                           const uint32_t *__restrict__ ccount,
                                                           const uint32_t *__restrict__ coff,
                                                           const uint32_t *__restrict__ clist, uint32_t ccap,
                                                           const float *__restrict__ dLdrgb,
                                                           const float *__restrict__ dLddepth,
                                                           float *__restrict__ dinst) {
    __shared__ float4 sA[256], sB[256], sC[256];
    __shared__ float sAcc[10][256];
    __shared__ uint32_t s_max;
    const uint32_t item = order ? order[blockIdx.x] : xcd_remap(blockIdx.x, gridDim.x);
    const int v = item / T, tile = item % T;
    const int tx = tile % ntx, ty = tile / ntx;
    const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
    const int px = tx * TW + lx, py = ty * TH + ly;
    const bool inside = px < W && py < H;
    const uint32_t start = ranges[2 * item], end = ranges[2 * item + 1];
    const int bx = (tx * TW) & ~31, by = (ty * TH) & ~31;
    const double ox = (double)bx, oy = (double)by;
    const float fx = (float)(px - bx) + 0.5f, fy = (float)(py - by) + 0.5f;
    const int64_t P = (int64_t)W * H;
    const int64_t pix = (int64_t)v * P + (int64_t)py * W + px;
    float Tr = 1.f, G0 = 0.f, G1 = 0.f, G2 = 0.f, GD = 0.f;
    int cur = -1;  // index into this pixel's list, walked down to 0
    uint32_t lbase = 0;
    if (inside) {
        Tr = Tfin[pix];
        G0 = dLdrgb[(int64_t)v * 3 * P + (int64_t)py * W + px];
        G1 = dLdrgb[(int64_t)v * 3 * P + P + (int64_t)py * W + px];
        G2 = dLdrgb[(int64_t)v * 3 * P + 2 * P + (int64_t)py * W + px];
        if (dLddepth) GD = dLddepth[pix];
        lbase = coff[pix];
        // a list that did not fit the capacity is incomplete: the caller must not pass one
        cur = lbase + ccount[pix] <= ccap ? (int)ccount[pix] - 1 : -1;
    }
    const gsr_camera &cam = cams[v];
    float S = Tr * (G0 * cam.bg[0] + G1 * cam.bg[1] + G2 * cam.bg[2]);
    // the deepest composited position over the tile's pixels bounds the batches
    uint32_t deep = cur >= 0 ? clist[lbase + cur] + 1 : 0u;
    if (threadIdx.x == 0) s_max = 0;
    for (int q = threadIdx.x; q < 2560; q += 256) (&sAcc[0][0])[q] = 0.f;
    __syncthreads();
    if (deep) atomicMax(&s_max, deep);
    __syncthreads();
    const uint32_t nl = min(s_max, end - start);
    for (uint32_t k = start + nl + threadIdx.x; k < end; k += 256) {
        float2 *rec = reinterpret_cast<float2 *>(dinst + (int64_t)inst_emit[k] * GSR_SPLAT_GRAD_FLOATS);
#pragma unroll
        for (int e = 0; e < 5; e++) rec[e] = make_float2(0.f, 0.f);
    }
    const float kap = (float)GSR_KAPPA;
    const float nln2 = -(float)GSR_LN2;
    uint32_t nextpos = cur >= 0 ? clist[lbase + cur] : 0u;
    for (int bend = (int)nl; bend > 0; bend -= 256) {
        const int b0 = bend > 256 ? bend - 256 : 0;
        const int cnt = bend - b0;
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            float4 A, B, C;
            stage_splat(splats, inst[start + b0 + threadIdx.x], ox, oy, A, B, C);
            sA[threadIdx.x] = A;
            sB[threadIdx.x] = B;
            sC[threadIdx.x] = C;
        }
        __syncthreads();
        while (cur >= 0 && nextpos >= (uint32_t)b0) {
            const int slot = (int)nextpos - b0;
            const float4 A = sA[slot], B = sB[slot], C = sC[slot];
            float dx, dy, u1, u2;
            const float Pw = blend_exponent(A, B.x, fx, fy, dx, dy, u1, u2);
            const float e2 = __builtin_amdgcn_exp2f(-Pw);
            const float ar = B.z * e2;
            const float a = fminf(ar, GSR_ALPHA_MAX);
            const float om = 1.0f - a;
            const float rom = __builtin_amdgcn_rcpf(om);
            const float Tb = Tr * rom;  // transmittance in front of it
            const float wgt = a * Tb;
            const float gsum = __builtin_fmaf(G0, C.x, __builtin_fmaf(G1, C.y, __builtin_fmaf(G2, C.z, GD * B.w)));
            const float dLda = __builtin_fmaf(Tb, gsum, -S * rom);
            float acc[10];
            const bool lin = ar <= GSR_ALPHA_MAX;
            const float dP = lin ? (nln2 * ar) * dLda : 0.f;
            acc[0] = -2.0f * dP * (A.z * u1);
            acc[1] = -2.0f * dP * __builtin_fmaf(A.w, u1, B.x * u2);
            acc[2] = dP * kap * dx * dx;
            acc[3] = dP * 2.0f * kap * dx * dy;
            acc[4] = dP * kap * dy * dy;
            acc[5] = lin ? dLda * e2 : 0.f;
            acc[6] = G0 * wgt;
            acc[7] = G1 * wgt;
            acc[8] = G2 * wgt;
            acc[9] = GD * wgt;
#pragma unroll
            for (int e = 0; e < 10; e++) atomicAdd(&sAcc[e][slot], acc[e]);
            S = __builtin_fmaf(wgt, gsum, S);
            Tr = Tb;
            cur--;
            nextpos = cur >= 0 ? clist[lbase + cur] : 0u;
        }
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            float2 *rec = reinterpret_cast<float2 *>(
                dinst + (int64_t)inst_emit[start + b0 + threadIdx.x] * GSR_SPLAT_GRAD_FLOATS);
#pragma unroll
            for (int e = 0; e < 5; e++) {
                rec[e] = make_float2(sAcc[2 * e][threadIdx.x], sAcc[2 * e + 1][threadIdx.x]);
                sAcc[2 * e][threadIdx.x] = 0.f;
                sAcc[2 * e + 1][threadIdx.x] = 0.f;
            }
        }
    }
}

}  // namespace gsr

using namespace gsr;

extern "C" size_t gsr_scan_ws_bytes(int64_t n);
extern "C" gsr_status gsr_scan_launch(const uint32_t *, int64_t, uint32_t *, uint32_t *, void *, hipStream_t);
extern "C" gsr_status gsr_fill_u32_launch(void *, uint32_t, int64_t, hipStream_t);

namespace {

struct SliceWs {
    uint32_t *tile_slices, *off, *count;
    void *scan;
    uint2 *info;
    float *tprod;
    float4 *part;
    uint2 *part2;
    uint32_t cap;
    size_t bytes;
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

// Every sliced tile holds len > kSplitMin = 8 kSliceLen instances, so its ceil(len / kSliceLen)
// slices number less than 1.125 len / kSliceLen: 1.125 capacity / kSliceLen + 1 always fit.
SliceWs slice_layout(void *base, int64_t VT, int64_t capacity) {
    SliceWs w{};
    const int64_t cap = 9 * (capacity > 0 ? capacity : 1) / (8 * (int64_t)kSliceLen) + 1;
    w.cap = (uint32_t)(cap < 0x7fffffff ? cap : 0x7fffffff);
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void *r = p ? p + off : nullptr;
        off += al256(bytes);
        return r;
    };
    w.tile_slices = static_cast<uint32_t *>(take((size_t)VT * 4));
    w.off = static_cast<uint32_t *>(take((size_t)VT * 4));
    w.count = static_cast<uint32_t *>(take(4));
    w.scan = take(gsr_scan_ws_bytes(VT));
    w.info = static_cast<uint2 *>(take((size_t)w.cap * sizeof(uint2)));
    w.tprod = static_cast<float *>(take((size_t)w.cap * kSubs * 256 * sizeof(float)));
    w.part = static_cast<float4 *>(take((size_t)w.cap * 256 * sizeof(float4)));
    w.part2 = static_cast<uint2 *>(take((size_t)w.cap * 256 * sizeof(uint2)));
    w.bytes = off;
    return w;
}

}  // namespace

extern "C" size_t gsr_render_fwd_ws_bytes(int V, const gsr_raster *r, int64_t capacity) {
    const int64_t T = ceil_div(r->width, r->tile_w) * ceil_div(r->height, r->tile_h);
    return slice_layout(nullptr, (int64_t)V * T, capacity).bytes;
}

// ws == NULL: every tile is composited whole (and n_contrib may be asked for); otherwise the
// tiles longer than kSliceLen are composited in depth slices (ncon must then be NULL).
extern "C" gsr_status gsr_render_fwd_launch(const gsr_splat *splats, const uint32_t *inst, const uint32_t *ranges,
                                            const uint32_t *order, const gsr_camera *cams, int V,
                                            const gsr_raster *r, float *rgb, float *depth, float *Tfin,
                                            uint32_t *last, uint32_t *ncon, int64_t capacity, void *ws,
                                            hipStream_t st) {
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    const int T = ntx * nty;
    const int nb = V * T;
    SliceArgs sl{};
    if (ws) {
        const SliceWs w = slice_layout(ws, nb, capacity);
        const int g = (int)(ceil_div(nb, 256) < 1024 ? ceil_div(nb, 256) : 1024);
        k_slice_count<<<g, 256, 0, st>>>(ranges, (uint32_t)nb, w.tile_slices);
        gsr_status s = gsr_scan_launch(w.tile_slices, nb, w.off, w.count, w.scan, st);
        if (s != GSR_OK) return s;
        k_slice_emit<<<g, 256, 0, st>>>(w.tile_slices, w.off, (uint32_t)nb, w.cap, w.info);
        sl = SliceArgs{w.tile_slices, w.info, w.count, w.tprod, w.part, w.part2, w.cap,
                       w.cap < 2048u ? w.cap : 2048u};
    }
#define GSR_RF(TW, TH)                                                                                            \
    do {                                                                                                          \
        if (sl.grid)                                                                                              \
            k_slice_prod<TW, TH><<<sl.grid, 256, 0, st>>>(splats, inst, ranges, r->width, r->height, ntx, T, sl); \
        if (ncon)                                                                                                 \
            k_render_fwd<TW, TH, false, true><<<nb + sl.grid, 256, 0, st>>>(                                      \
                splats, inst, ranges, order, cams, r->width, r->height, ntx, T, rgb, depth, Tfin, last, ncon,     \
                nullptr, nullptr, 0u, sl);                                                                        \
        else                                                                                                      \
            k_render_fwd<TW, TH, false><<<nb + sl.grid, 256, 0, st>>>(splats, inst, ranges, order, cams, r->width, \
                                                                      r->height, ntx, T, rgb, depth, Tfin, last,  \
                                                                      nullptr, nullptr, nullptr, 0u, sl);         \
        if (sl.grid)                                                                                              \
            k_slice_merge<TW, TH><<<sl.grid, 256, 0, st>>>(ranges, cams, r->width, r->height, ntx, T, sl, rgb,    \
                                                           depth, Tfin, last);                                    \
    } while (0)
    if (r->tile_w == 16) GSR_RF(16, 16);
    else if (r->tile_w == 8) GSR_RF(8, 32);
    else GSR_RF(32, 8);
#undef GSR_RF
    return last_launch();
}

// Workspace of the fused step: the depth-slice workspace, then per view-tile loss sums (double),
// then the work-queue counter and per view-tile slice completion counters.
extern "C" size_t gsr_render_step_ws_bytes(int V, const gsr_raster *r, int64_t capacity) {
    const int64_t VT = (int64_t)V * ceil_div(r->width, r->tile_w) * ceil_div(r->height, r->tile_h);
    return slice_layout(nullptr, VT, capacity).bytes + al256((size_t)VT * 8) + al256((size_t)(VT + 1) * 4);
}

namespace {
// Resident workgroups of a kernel on the current device (the persistent grid).
int persistent_grid(const void *kernel) {
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, 256, 0) != hipSuccess) return 0;
    return ncu * (per > 0 ? per : 1);
}
}  // namespace

extern "C" gsr_status gsr_render_step_launch(const gsr_splat *splats, const uint32_t *inst, const uint32_t *inst_emit,
                                             const uint32_t *ranges, const uint32_t *order, const gsr_camera *cams,
                                             int V, const gsr_raster *r, const float *trgb, const float *tdepth,
                                             const int32_t *tidx, float lam, float *rgb, float *depth, float *Tfin,
                                             uint32_t *last, double *loss, float *dinst, int64_t capacity, void *ws,
                                             hipStream_t st) {
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    const int T = ntx * nty;
    const int nb = V * T;
    const SliceWs w = slice_layout(ws, nb, capacity);
    double *item_loss = reinterpret_cast<double *>(static_cast<char *>(ws) + w.bytes);
    uint32_t *counters = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + w.bytes + al256((size_t)nb * 8));
    const int g = (int)(ceil_div(nb, 256) < 1024 ? ceil_div(nb, 256) : 1024);
    k_slice_count<<<g, 256, 0, st>>>(ranges, (uint32_t)nb, w.tile_slices);
    gsr_status s = gsr_scan_launch(w.tile_slices, nb, w.off, w.count, w.scan, st);
    if (s != GSR_OK) return s;
    k_slice_emit<<<g, 256, 0, st>>>(w.tile_slices, w.off, (uint32_t)nb, w.cap, w.info);
    s = gsr_fill_u32_launch(counters, 0u, (int64_t)nb + 1, st);
    if (s != GSR_OK) return s;
    const SliceArgs sl{w.tile_slices, w.info, w.count, w.tprod, w.part, w.part2, w.cap, w.cap < 2048u ? w.cap : 2048u};
    const StepArgs a{trgb, tdepth, tidx, lam, item_loss, counters, counters + 1};
#define GSR_RSTEP(TW, TH)                                                                                          \
    do {                                                                                                           \
        const int grid = persistent_grid(reinterpret_cast<const void *>(&k_render_step<TW, TH>));                 \
        if (grid <= 0) return GSR_E_HIP;                                                                          \
        k_slice_prod<TW, TH><<<sl.grid, 256, 0, st>>>(splats, inst, ranges, r->width, r->height, ntx, T, sl);      \
        k_render_step<TW, TH><<<grid, 256, 0, st>>>(splats, inst, inst_emit, ranges, order, cams, r->width,         \
                                                    r->height, ntx, T, (uint32_t)nb, rgb, depth, Tfin, last, dinst, \
                                                    sl, a);                                                        \
    } while (0)
    if (r->tile_w == 16) GSR_RSTEP(16, 16);
    else if (r->tile_w == 8) GSR_RSTEP(8, 32);
    else GSR_RSTEP(32, 8);
#undef GSR_RSTEP
    k_step_loss<<<1, 1024, 0, st>>>(item_loss, (uint32_t)nb, 1.0 / ((double)r->width * r->height), loss);
    return last_launch();
}

extern "C" size_t gsr_render_bwd_l1_ws_bytes(int V, const gsr_raster *r) {
    return al256((size_t)V * ceil_div(r->width, r->tile_w) * ceil_div(r->height, r->tile_h) * 8);
}

extern "C" gsr_status gsr_render_bwd_l1_launch(const gsr_splat *splats, const uint32_t *inst,
                                               const uint32_t *inst_emit, const uint32_t *ranges,
                                               const uint32_t *order, const gsr_camera *cams, int V,
                                               const gsr_raster *r, const float *rgb, const float *depth,
                                               const float *Tfin, const uint32_t *last, const float *trgb,
                                               const float *tdepth, const int32_t *tidx, float lam, double *loss,
                                               float *dinst, void *ws, void *fwd_ws, int64_t capacity,
                                               hipStream_t st) {
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    const int T = ntx * nty;
    const int nb = V * T;
    double *item_loss = static_cast<double *>(ws);
    const StepArgs a{trgb, tdepth, tidx, lam, item_loss, nullptr, nullptr};
    // the long tiles run in the depth slices of the sliced forward that produced the images
    SliceArgs sl{};
    if (fwd_ws) {
        const SliceWs w = slice_layout(fwd_ws, nb, capacity);
        sl = SliceArgs{w.tile_slices, w.info, w.count, w.tprod, w.part, w.part2, w.cap, w.cap < 2048u ? w.cap : 2048u};
    }
#define GSR_RBL(TW, TH)                                                                                         \
    k_render_bwd_l1<TW, TH><<<nb + sl.grid, 256, 0, st>>>(splats, inst, inst_emit, ranges, order, cams, r->width, \
                                                          r->height, ntx, T, rgb, depth, Tfin, last, dinst, a, sl)
    if (r->tile_w == 16) GSR_RBL(16, 16);
    else if (r->tile_w == 8) GSR_RBL(8, 32);
    else GSR_RBL(32, 8);
#undef GSR_RBL
    k_step_loss<<<1, 1024, 0, st>>>(item_loss, (uint32_t)nb, 1.0 / ((double)r->width * r->height), loss);
    return last_launch();
}

// Second pass of the stored-contributor forward: the per-pixel lists.
extern "C" gsr_status gsr_render_store_launch(const gsr_splat *splats, const uint32_t *inst, const uint32_t *ranges,
                                             const uint32_t *order, const gsr_camera *cams, int V,
                                             const gsr_raster *r, const uint32_t *coff, uint32_t *clist,
                                             uint32_t ccap, hipStream_t st) {
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    const int T = ntx * nty;
    const int nb = V * T;
#define GSR_RS(TW, TH)                                                                                        \
    k_render_fwd<TW, TH, true><<<nb, 256, 0, st>>>(splats, inst, ranges, order, cams, r->width, r->height, ntx, T, \
                                                   nullptr, nullptr, nullptr, nullptr, nullptr, coff, clist, ccap, \
                                                   SliceArgs{})
    if (r->tile_w == 16) GSR_RS(16, 16);
    else if (r->tile_w == 8) GSR_RS(8, 32);
    else GSR_RS(32, 8);
#undef GSR_RS
    return last_launch();
}

extern "C" gsr_status gsr_render_bwd_launch(const gsr_splat *splats, const uint32_t *inst, const uint32_t *inst_emit,
                                            const uint32_t *ranges, const uint32_t *order, const gsr_camera *cams,
                                            int V, const gsr_raster *r, const float *Tfin, const uint32_t *last,
                                            const float *dLdrgb, const float *dLddepth, float *dinst,
                                            void *fwd_ws, int64_t capacity, hipStream_t st) {
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    const int T = ntx * nty;
    const int nb = V * T;
    // the long tiles run in the depth slices of the sliced forward that produced T_final and last
    SliceArgs sl{};
    if (fwd_ws) {
        const SliceWs w = slice_layout(fwd_ws, nb, capacity);
        sl = SliceArgs{w.tile_slices, w.info, w.count, w.tprod, w.part, w.part2, w.cap, w.cap < 2048u ? w.cap : 2048u};
    }
#define GSR_RB(TW, TH)                                                                                            \
    k_render_bwd<TW, TH><<<nb + sl.grid, 256, 0, st>>>(splats, inst, inst_emit, ranges, order, cams, r->width,     \
                                                       r->height, ntx, T, Tfin, last, dLdrgb, dLddepth, dinst, sl)
    if (r->tile_w == 16) GSR_RB(16, 16);
    else if (r->tile_w == 8) GSR_RB(8, 32);
    else GSR_RB(32, 8);
#undef GSR_RB
    return last_launch();
}

extern "C" gsr_status gsr_render_bwd_stored_launch(const gsr_splat *splats, const uint32_t *inst,
                                                   const uint32_t *inst_emit, const uint32_t *ranges,
                                                   const uint32_t *order, const gsr_camera *cams, int V,
                                                   const gsr_raster *r, const float *Tfin, const uint32_t *ccount,
                                                   const uint32_t *coff, const uint32_t *clist, uint32_t ccap,
                                                   const float *dLdrgb, const float *dLddepth, float *dinst,
                                                   hipStream_t st) {
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    const int T = ntx * nty;
    const int nb = V * T;
#define GSR_RBS(TW, TH)                                                                                          \
    k_render_bwd_stored<TW, TH><<<nb, 256, 0, st>>>(splats, inst, inst_emit, ranges, order, cams, r->width,      \
                                                    r->height, ntx, T, Tfin, ccount, coff, clist, ccap, dLdrgb,    \
                                                    dLddepth, dinst)
    if (r->tile_w == 16) GSR_RBS(16, 16);
    else if (r->tile_w == 8) GSR_RBS(8, 32);
    else GSR_RBS(32, 8);
#undef GSR_RBS
    return last_launch();
}

