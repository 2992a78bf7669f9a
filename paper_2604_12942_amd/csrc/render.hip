// Front-to-back alpha compositing of colour and depth (Eq. 8) and its exact backward.
//
// One 256-lane workgroup (four wave64s) per (view, screen tile); one pixel per lane.  The tile's
// depth-ordered instances are staged through LDS in batches of 256: each lane gathers one
// projected splat (48 B), re-centres its double-precision mean near the tile and stores
// the float32 fields the blend loop needs; every lane then walks the batch reading the staged
// values as LDS broadcasts.  The blend exponent is evaluated in the whitened form
// |L^T D|^2 (L the Cholesky factor of (log2(e)/2) Q): two fused products per pair and no
// cancellation for thin ellipses, and exp2 is the hardware v_exp_f32.
#include "gsr_internal.h"

namespace gsr {

struct Staged {
    float4 A;  // mx, my (mean relative to the 32-aligned block origin), l11, l21
    float4 B;  // l22, cut = log2(255 o), o, z
    float4 C;  // r, g, b, (unused)
};

__device__ __forceinline__ void stage_splat(const gsr_splat *__restrict__ splats, uint32_t gid, double ox, double oy,
                                            float4 &A, float4 &B, float4 &C) {
    const double2 uv = *reinterpret_cast<const double2 *>(splats + gid);
    const float4 f1 = *(reinterpret_cast<const float4 *>(splats + gid) + 1);
    const float4 f2 = *(reinterpret_cast<const float4 *>(splats + gid) + 2);
    A = make_float4((float)(uv.x - ox), (float)(uv.y - oy), f1.x, f1.y);
    B = make_float4(f1.z, __log2f(255.0f * f1.w), f1.w, f2.x);
    C = make_float4(f2.y, f2.z, f2.w, 0.0f);
}

// Whitened exponent at the pixel centre (fx, fy) in tile coordinates.  Forward and backward
// both call this, so their contribute / skip decisions are bit-identical.
__device__ __forceinline__ float blend_exponent(const float4 &A, float l22, float fx, float fy, float &dx, float &dy,
                                                float &u1, float &u2) {
    dx = fx - A.x;
    dy = fy - A.y;
    u1 = __builtin_fmaf(A.z, dx, A.w * dy);
    u2 = l22 * dy;
    return __builtin_fmaf(u1, u1, u2 * u2);
}

template <int TW, int TH>
__global__ __launch_bounds__(256) void k_render_fwd(const gsr_splat *__restrict__ splats,
                                                    const uint32_t *__restrict__ inst,
                                                    const uint32_t *__restrict__ ranges,
                                                    const gsr_camera *__restrict__ cams, int W, int H, int ntx,
                                                    int T, float *__restrict__ rgb, float *__restrict__ depth,
                                                    float *__restrict__ Tfin, uint32_t *__restrict__ last,
                                                    uint32_t *__restrict__ ncon) {
    static_assert(TW * TH == 256, "one pixel per lane");
    __shared__ float4 sA[256], sB[256], sC[256];
    const uint32_t item = xcd_remap(blockIdx.x, gridDim.x);
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
    float Tr = 1.0f, c0 = 0.f, c1 = 0.f, c2 = 0.f, dd = 0.f;
    uint32_t lst = 0, nc = 0;
    bool done = !inside;
    for (uint32_t b = start; b < end; b += 256) {
        if (__syncthreads_count(!done) == 0) break;
        const uint32_t e = b + threadIdx.x;
        if (e < end) {
            float4 A, B, C;
            stage_splat(splats, inst[e], ox, oy, A, B, C);
            sA[threadIdx.x] = A;
            sB[threadIdx.x] = B;
            sC[threadIdx.x] = C;
        }
        __syncthreads();
        const int cnt = (int)min(256u, end - b);
        for (int j = 0; j < cnt && !done; j++) {
            const float4 A = sA[j];
            const float4 B = sB[j];
            float dx, dy, u1, u2;
            const float P = blend_exponent(A, B.x, fx, fy, dx, dy, u1, u2);
            if (P > B.y) continue;
            const float ar = B.z * __builtin_amdgcn_exp2f(-P);
            const float a = fminf(ar, GSR_ALPHA_MAX);
            const float Tn = Tr * (1.0f - a);
            if (Tn < GSR_T_MIN) {
                done = true;
                break;
            }
            const float wgt = a * Tr;
            const float4 C = sC[j];
            c0 = __builtin_fmaf(wgt, C.x, c0);
            c1 = __builtin_fmaf(wgt, C.y, c1);
            c2 = __builtin_fmaf(wgt, C.z, c2);
            dd = __builtin_fmaf(wgt, B.w, dd);
            Tr = Tn;
            lst = b - start + j + 1;
            nc++;
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

template <int TW, int TH>
__global__ __launch_bounds__(256) void k_render_bwd(const gsr_splat *__restrict__ splats,
                                                    const uint32_t *__restrict__ inst,
                                                    const uint32_t *__restrict__ ranges,
                                                    const gsr_camera *__restrict__ cams, int W, int H, int ntx,
                                                    int T, const float *__restrict__ Tfin,
                                                    const uint32_t *__restrict__ last,
                                                    const float *__restrict__ dLdrgb,
                                                    const float *__restrict__ dLddepth,
                                                    float *__restrict__ dsplat) {
    __shared__ float4 sA[256], sB[256], sC[256];
    __shared__ uint32_t sG[256];
    __shared__ uint32_t s_max;
    const uint32_t item = xcd_remap(blockIdx.x, gridDim.x);
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
    const int64_t pix = (int64_t)py * W + px;
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
    // S = sum over later contributors of w_j (G . c_j + GD z_j) plus the background term
    float S = Tr * (G0 * cam.bg[0] + G1 * cam.bg[1] + G2 * cam.bg[2]);
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    if (mylast) atomicMax(&s_max, mylast);
    __syncthreads();
    const uint32_t nl = min(s_max, end - start);
    const float kap = (float)GSR_KAPPA;
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
        for (int j = cnt - 1; j >= 0; j--) {
            float g[10];
#pragma unroll
            for (int e = 0; e < 10; e++) g[e] = 0.f;
            bool contrib = false;
            if ((uint32_t)(b0 + j) < mylast) {
                const float4 A = sA[j];
                const float4 B = sB[j];
                float dx, dy, u1, u2;
                const float Pw = blend_exponent(A, B.x, fx, fy, dx, dy, u1, u2);
                if (Pw <= B.y) {
                    contrib = true;
                    const float e2 = __builtin_amdgcn_exp2f(-Pw);
                    const float ar = B.z * e2;
                    const float a = fminf(ar, GSR_ALPHA_MAX);
                    const float om = 1.0f - a;
                    const float Tk = Tr / om;  // transmittance in front of this contributor
                    const float wgt = a * Tk;
                    const float4 C = sC[j];
                    const float gsum = G0 * C.x + G1 * C.y + G2 * C.z + GD * B.w;
                    const float dLda = Tk * gsum - S / om;
                    S = __builtin_fmaf(wgt, gsum, S);
                    Tr = Tk;
                    g[6] = G0 * wgt;
                    g[7] = G1 * wgt;
                    g[8] = G2 * wgt;
                    g[9] = GD * wgt;
                    if (ar <= GSR_ALPHA_MAX) {
                        // alpha_raw = o 2^-P: d/dP = -ln2 alpha_raw, d/do = 2^-P
                        const float dP = -(float)GSR_LN2 * ar * dLda;
                        g[0] = -2.0f * dP * (A.z * u1);
                        g[1] = -2.0f * dP * (A.w * u1 + B.x * u2);
                        g[2] = dP * kap * dx * dx;
                        g[3] = dP * 2.0f * kap * dx * dy;
                        g[4] = dP * kap * dy * dy;
                        g[5] = dLda * e2;
                    }
                }
            }
            if (__ballot(contrib)) {
                const uint32_t gid = sG[j];
#pragma unroll
                for (int e = 0; e < 10; e++) {
                    const float s = wave_sum(g[e]);
                    if (__lane_id() == 0 && s != 0.f) atomicAdd(dsplat + (int64_t)gid * 10 + e, s);
                }
            }
        }
    }
}

}  // namespace gsr

using namespace gsr;

extern "C" gsr_status gsr_render_fwd_launch(const gsr_splat *splats, const uint32_t *inst, const uint32_t *ranges,
                                            const gsr_camera *cams, int V, const gsr_raster *r, float *rgb,
                                            float *depth, float *Tfin, uint32_t *last, uint32_t *ncon,
                                            hipStream_t st) {
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    const int T = ntx * nty;
    const int nb = V * T;
#define GSR_RF(TW, TH) \
    k_render_fwd<TW, TH><<<nb, 256, 0, st>>>(splats, inst, ranges, cams, r->width, r->height, ntx, T, rgb, depth, Tfin, last, \
                                             ncon)
    if (r->tile_w == 16) GSR_RF(16, 16);
    else if (r->tile_w == 8) GSR_RF(8, 32);
    else GSR_RF(32, 8);
#undef GSR_RF
    return last_launch();
}

extern "C" gsr_status gsr_render_bwd_launch(const gsr_splat *splats, const uint32_t *inst, const uint32_t *ranges,
                                            const gsr_camera *cams, int V, const gsr_raster *r, const float *Tfin,
                                            const uint32_t *last, const float *dLdrgb, const float *dLddepth,
                                            float *dsplat, hipStream_t st) {
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    const int T = ntx * nty;
    const int nb = V * T;
#define GSR_RB(TW, TH)                                                                                        \
    k_render_bwd<TW, TH><<<nb, 256, 0, st>>>(splats, inst, ranges, cams, r->width, r->height, ntx, T, Tfin, last, \
                                             dLdrgb, dLddepth, dsplat)
    if (r->tile_w == 16) GSR_RB(16, 16);
    else if (r->tile_w == 8) GSR_RB(8, 32);
    else GSR_RB(32, 8);
#undef GSR_RB
    return last_launch();
}
