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

// Whitened exponent at the pixel centre (fx, fy) (32x32-block coordinates).  Forward and
// backward both call this, so their contribute / skip decisions are bit-identical.
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

template <int TW, int TH>
__global__ __launch_bounds__(256) void k_render_fwd(const gsr_splat *__restrict__ splats,
                                                    const uint32_t *__restrict__ inst,
                                                    const uint32_t *__restrict__ ranges,
                                                    const uint32_t *__restrict__ order,
                                                    const gsr_camera *__restrict__ cams, int W, int H, int ntx,
                                                    int T, float *__restrict__ rgb, float *__restrict__ depth,
                                                    float *__restrict__ Tfin, uint32_t *__restrict__ last,
                                                    uint32_t *__restrict__ ncon) {
    static_assert(TW * TH == 256, "one pixel per lane");
    __shared__ float4 sA[256], sB[256], sC[256];
    const uint32_t item = order ? order[blockIdx.x] : xcd_remap(blockIdx.x, gridDim.x);
    const int v = item / T, tile = item % T;
    const int tx = tile % ntx, ty = tile / ntx;
    const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
    const int px = tx * TW + lx, py = ty * TH + ly;
    const bool inside = px < W && py < H;
    const uint32_t start = ranges[2 * item], end = ranges[2 * item + 1];
    // means are re-centred on the 32x32-aligned block holding the tile: the same origin for
    // every tile shape, so images are bit-identical across 16x16, 8x32 and 32x8 tiles
    const int bx = (tx * TW) & ~31, by = (ty * TH) & ~31;
    const double ox = (double)bx, oy = (double)by;
    const float fx = (float)(px - bx) + 0.5f, fy = (float)(py - by) + 0.5f;
    const int w = threadIdx.x >> 6;
    float wx0, wx1, wy0, wy1;
    wave_box<TW>(tx * TW - bx, ty * TH - by, w, wx0, wx1, wy0, wy1);
    float Tr = 1.0f, c0 = 0.f, c1 = 0.f, c2 = 0.f, dd = 0.f;
    uint32_t lst = 0, nc = 0;
    bool done = !inside;
    for (uint32_t b = start; b < end; b += 256) {
        if (__syncthreads_count(!done) == 0) break;
        const uint32_t e = b + threadIdx.x;
        const int cnt = (int)min(256u, end - b);
        if (e < end) {
            float4 A, B, C;
            stage_splat(splats, inst[e], ox, oy, A, B, C);
            sA[threadIdx.x] = A;
            sB[threadIdx.x] = B;
            sC[threadIdx.x] = C;
        }
        __syncthreads();
        if (__ballot(!done) == 0) continue;  // the whole wave has terminated
        // which staged Gaussians reach this wave's pixels
        uint64_t rel[4];
#pragma unroll
        for (int g = 0; g < 4; g++) {
            const int slot = g * 64 + __lane_id();
            bool r = false;
            if (slot < cnt) r = ellipse_meets_box(sA[slot], sB[slot], wx0, wx1, wy0, wy1);
            rel[g] = __ballot(r);
        }
        const uint32_t pos0 = b - start + 1;
#pragma unroll
        for (int g = 0; g < 4; g++) {
            uint64_t m = rel[g];
            while (m) {
                const int j = g * 64 + __builtin_ctzll(m);
                m &= m - 1;
                const float4 A = sA[j];
                const float4 B = sB[j];
                float dx, dy, u1, u2;
                const float P = blend_exponent(A, B.x, fx, fy, dx, dy, u1, u2);
                // branch-free: non-contributing lanes blend with weight exactly 0
                const bool cont = (P <= B.y) && !done;
                const float ar = B.z * __builtin_amdgcn_exp2f(-P);
                const float a0 = cont ? fminf(ar, GSR_ALPHA_MAX) : 0.0f;
                const bool term = (Tr * (1.0f - a0)) < GSR_T_MIN;
                done = done || term;
                const float a = term ? 0.0f : a0;
                const float wgt = a * Tr;
                const float4 C = sC[j];
                c0 = __builtin_fmaf(wgt, C.x, c0);
                c1 = __builtin_fmaf(wgt, C.y, c1);
                c2 = __builtin_fmaf(wgt, C.z, c2);
                dd = __builtin_fmaf(wgt, B.w, dd);
                Tr = Tr * (1.0f - a);
                const bool used = a > 0.0f;
                lst = used ? pos0 + (uint32_t)j : lst;
                nc += used ? 1u : 0u;
            }
        }
    }
    if (!inside) return;
    const gsr_camera &cam = cams[v];
    const int64_t P = (int64_t)W * H;
    const int64_t pix = (int64_t)py * W + px;
    rgb[(int64_t)v * 3 * P + pix] = __builtin_fmaf(Tr, cam.bg[0], c0);
    rgb[(int64_t)v * 3 * P + P + pix] = __builtin_fmaf(Tr, cam.bg[1], c1);
    rgb[(int64_t)v * 3 * P + 2 * P + pix] = __builtin_fmaf(Tr, cam.bg[2], c2);
    depth[(int64_t)v * P + pix] = dd;
    Tfin[(int64_t)v * P + pix] = Tr;
    last[(int64_t)v * P + pix] = lst;
    if (ncon) ncon[(int64_t)v * P + pix] = nc;
}

// ---- wave64 inclusive scans over lane order (DPP row shifts, then row broadcasts) -------------
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_or(float src, float ident) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(ident), __float_as_int(src), CTRL, ROWS, 0xf,
                                                      false));
}
__device__ __forceinline__ float wave_incl_prod(float v) {
    v *= dpp_or<0x111, 0xf>(v, 1.0f);  // row_shr:1
    v *= dpp_or<0x112, 0xf>(v, 1.0f);  // row_shr:2
    v *= dpp_or<0x114, 0xf>(v, 1.0f);  // row_shr:4
    v *= dpp_or<0x118, 0xf>(v, 1.0f);  // row_shr:8
    v *= dpp_or<0x142, 0xa>(v, 1.0f);  // row_bcast:15 into rows 1 and 3
    v *= dpp_or<0x143, 0xc>(v, 1.0f);  // row_bcast:31 into rows 2 and 3
    return v;
}
__device__ __forceinline__ float wave_incl_sum(float v) {
    v += dpp_or<0x111, 0xf>(v, 0.0f);
    v += dpp_or<0x112, 0xf>(v, 0.0f);
    v += dpp_or<0x114, 0xf>(v, 0.0f);
    v += dpp_or<0x118, 0xf>(v, 0.0f);
    v += dpp_or<0x142, 0xa>(v, 0.0f);
    v += dpp_or<0x143, 0xc>(v, 0.0f);
    return v;
}
__device__ __forceinline__ float rdl(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ float wrl(float v, int lane, float old) { return __lane_id() == lane ? v : old; }

// Backward, Gaussian-major.  The tile's instances up to the deepest pixel's last contributor are
// staged back to front in batches of 256.  Each wave compacts the batch to the Gaussians that
// reach its pixel sub-rectangle and cuts them, deepest first, into chunks of 64: lane l holds the
// l-th deepest.  For each of the wave's 64 pixels every lane evaluates its Gaussian; a wave-wide
// inclusive product scan of (1 - a) recovers the transmittance in front of each Gaussian from the
// pixel's transmittance behind the chunk, and an inclusive sum scan of w (dL/dC . c + dL/dD z)
// gives what lies behind it.  Gradients accumulate in registers across pixels, then in LDS across
// waves (ds_add_f32 per staged slot), and leave with one global atomic per (tile, Gaussian,
// component).
template <int TW, int TH>
__global__ __launch_bounds__(256) void k_render_bwd(const gsr_splat *__restrict__ splats,
                                                    const uint32_t *__restrict__ inst,
                                                    const uint32_t *__restrict__ ranges,
                                                    const uint32_t *__restrict__ order,
                                                    const gsr_camera *__restrict__ cams, int W, int H, int ntx,
                                                    int T, const float *__restrict__ Tfin,
                                                    const uint32_t *__restrict__ last,
                                                    const float *__restrict__ dLdrgb,
                                                    const float *__restrict__ dLddepth,
                                                    float *__restrict__ dsplat) {
    __shared__ float4 sA[256], sB[256], sC[256];
    __shared__ uint32_t sG[256];
    __shared__ float sAcc[10][256];
    __shared__ uint8_t sList[4][256];
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
    // per-pixel state, one pixel per lane (read by the wave with readlane)
    const float fx = (float)(px - bx) + 0.5f, fy = (float)(py - by) + 0.5f;
    const int64_t P = (int64_t)W * H;
    const int64_t pix = (int64_t)py * W + px;
    const int lane = __lane_id(), w = threadIdx.x >> 6;
    float wx0, wx1, wy0, wy1;
    wave_box<TW>(tx * TW - bx, ty * TH - by, w, wx0, wx1, wy0, wy1);
    float Tr = 1.f, G0 = 0.f, G1 = 0.f, G2 = 0.f, GD = 0.f;
    uint32_t mylast = 0;
    if (inside) {
        Tr = Tfin[(int64_t)v * P + pix];
        mylast = last[(int64_t)v * P + pix];
        G0 = dLdrgb[(int64_t)v * 3 * P + pix];
        G1 = dLdrgb[(int64_t)v * 3 * P + P + pix];
        G2 = dLdrgb[(int64_t)v * 3 * P + 2 * P + pix];
        if (dLddepth) GD = dLddepth[(int64_t)v * P + pix];
    }
    const gsr_camera &cam = cams[v];
    // S = sum over contributors behind of w_j (dL/dC . c_j + dL/dD z_j) plus the background term
    float S = Tr * (G0 * cam.bg[0] + G1 * cam.bg[1] + G2 * cam.bg[2]);
    if (threadIdx.x == 0) s_max = 0;
    for (int q = threadIdx.x; q < 2560; q += 256) (&sAcc[0][0])[q] = 0.f;
    __syncthreads();
    if (mylast) atomicMax(&s_max, mylast);
    // the deepest last contributor of this wave's pixels
    uint32_t wmax = mylast;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wmax = max(wmax, (uint32_t)__shfl_xor((int)wmax, off));
    __syncthreads();
    const uint32_t nl = min(s_max, end - start);
    const float kap = (float)GSR_KAPPA;
    const float ln2 = (float)GSR_LN2;
    for (int bend = (int)nl; bend > 0; bend -= 256) {
        const int b0 = bend > 256 ? bend - 256 : 0;
        const int cnt = bend - b0;
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const uint32_t gid = inst[start + b0 + threadIdx.x];
            float4 A, B, C;
            stage_splat(splats, gid, ox, oy, A, B, C);
            sA[threadIdx.x] = A;
            sB[threadIdx.x] = B;
            sC[threadIdx.x] = C;
            sG[threadIdx.x] = gid;
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
        for (int c0 = 0; c0 < nw; c0 += 64) {
            const int idx = c0 + lane;
            const bool gvalid = idx < nw;
            const int slot = gvalid ? sList[w][idx] : 0;
            const float4 A = gvalid ? sA[slot] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 B = gvalid ? sB[slot] : make_float4(0.f, -1.f, 0.f, 0.f);
            const float4 C = gvalid ? sC[slot] : make_float4(0.f, 0.f, 0.f, 0.f);
            const uint32_t pos = (uint32_t)(b0 + slot);
            // frontmost position of the chunk: the last valid lane
            const int lastlane = (nw - c0 < 64 ? nw - c0 : 64) - 1;
            const uint32_t cfront = (uint32_t)__builtin_amdgcn_readlane((int)pos, lastlane);
            float acc[10];
#pragma unroll
            for (int e = 0; e < 10; e++) acc[e] = 0.f;
            for (int p = 0; p < 64; p++) {
                const uint32_t lastp = (uint32_t)__builtin_amdgcn_readlane((int)mylast, p);
                if (cfront >= lastp) continue;
                const float pfx = rdl(fx, p), pfy = rdl(fy, p);
                float dx, dy, u1, u2;
                const float Pw = blend_exponent(A, B.x, pfx, pfy, dx, dy, u1, u2);
                const bool act = gvalid && pos < lastp && Pw <= B.y;
                if (__ballot(act) == 0) continue;  // no Gaussian of the chunk reaches this pixel
                const float e2 = act ? __builtin_amdgcn_exp2f(-Pw) : 0.f;
                const float ar = B.z * e2;
                const float a = fminf(ar, GSR_ALPHA_MAX);
                const float om = 1.0f - a;
                const float Te = rdl(Tr, p), Se = rdl(S, p);
                const float g0 = rdl(G0, p), g1 = rdl(G1, p), g2 = rdl(G2, p), gd = rdl(GD, p);
                const float Pt = wave_incl_prod(om);
                const float Tb = Te * __builtin_amdgcn_rcpf(Pt);  // transmittance in front of it
                const float wgt = a * Tb;
                const float gsum = g0 * C.x + g1 * C.y + g2 * C.z + gd * B.w;
                const float wg = wgt * gsum;
                const float incl = wave_incl_sum(wg);
                const float Sa = Se + (incl - wg);  // everything behind it
                const float dLda = Tb * gsum - Sa * __builtin_amdgcn_rcpf(om);
                if (act) {
                    acc[6] = __builtin_fmaf(g0, wgt, acc[6]);
                    acc[7] = __builtin_fmaf(g1, wgt, acc[7]);
                    acc[8] = __builtin_fmaf(g2, wgt, acc[8]);
                    acc[9] = __builtin_fmaf(gd, wgt, acc[9]);
                    if (ar <= GSR_ALPHA_MAX) {
                        // alpha_raw = o 2^-P: d/dP = -ln2 alpha_raw, d/do = 2^-P
                        const float dP = -ln2 * ar * dLda;
                        acc[0] -= 2.0f * dP * (A.z * u1);
                        acc[1] -= 2.0f * dP * (A.w * u1 + B.x * u2);
                        acc[2] += dP * kap * dx * dx;
                        acc[3] += dP * 2.0f * kap * dx * dy;
                        acc[4] += dP * kap * dy * dy;
                        acc[5] = __builtin_fmaf(dLda, e2, acc[5]);
                    }
                }
                // the pixel's state in front of this chunk (inactive lanes carry a = 0)
                Tr = wrl(rdl(Tb, 63), p, Tr);
                S = wrl(Se + rdl(incl, 63), p, S);
            }
            if (gvalid) {
#pragma unroll
                for (int e = 0; e < 10; e++)
                    if (acc[e] != 0.f) atomicAdd(&sAcc[e][slot], acc[e]);
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < 2560; q += 256) {
            const int e = q >> 8, sl = q & 255;
            const float sum = sAcc[e][sl];
            if (sum != 0.f) {
                atomicAdd(dsplat + (int64_t)sG[sl] * 10 + e, sum);
                sAcc[e][sl] = 0.f;
            }
        }
    }
}

}  // namespace gsr

using namespace gsr;

extern "C" gsr_status gsr_render_fwd_launch(const gsr_splat *splats, const uint32_t *inst, const uint32_t *ranges,
                                            const uint32_t *order, const gsr_camera *cams, int V,
                                            const gsr_raster *r, float *rgb, float *depth, float *Tfin,
                                            uint32_t *last, uint32_t *ncon, hipStream_t st) {
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    const int T = ntx * nty;
    const int nb = V * T;
#define GSR_RF(TW, TH)                                                                                               \
    k_render_fwd<TW, TH><<<nb, 256, 0, st>>>(splats, inst, ranges, order, cams, r->width, r->height, ntx, T, rgb, \
                                             depth, Tfin, last, ncon)
    if (r->tile_w == 16) GSR_RF(16, 16);
    else if (r->tile_w == 8) GSR_RF(8, 32);
    else GSR_RF(32, 8);
#undef GSR_RF
    return last_launch();
}

extern "C" gsr_status gsr_render_bwd_launch(const gsr_splat *splats, const uint32_t *inst, const uint32_t *ranges,
                                            const uint32_t *order, const gsr_camera *cams, int V,
                                            const gsr_raster *r, const float *Tfin, const uint32_t *last,
                                            const float *dLdrgb, const float *dLddepth, float *dsplat,
                                            hipStream_t st) {
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    const int T = ntx * nty;
    const int nb = V * T;
#define GSR_RB(TW, TH)                                                                                          \
    k_render_bwd<TW, TH><<<nb, 256, 0, st>>>(splats, inst, ranges, order, cams, r->width, r->height, ntx, T, \
                                             Tfin, last, dLdrgb, dLddepth, dsplat)
    if (r->tile_w == 16) GSR_RB(16, 16);
    else if (r->tile_w == 8) GSR_RB(8, 32);
    else GSR_RB(32, 8);
#undef GSR_RB
    return last_launch();
}
