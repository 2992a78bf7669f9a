// Supervision masks and the full training loss of Sec. III-C: the support mask from the
// accumulated opacity and its disk erosion (Eq. 7), and Eq. 9 with the masked L1 colour and
// depth terms (Eq. 10, 12) and the SSIM term on the mask-restricted images (Eq. 11).
//
// All of it is image-space work over V x H x W pixels.  The L1 terms are one coalesced stream.
// SSIM is non-local (11 x 11 window), so it takes two tiled kernels: the forward stages a
// 42 x 42 block of both images in LDS (a 32 x 32 output tile and its 5-pixel frame), filters the
// five window moments separably and writes, per pixel and channel, the three derivatives of the
// loss with respect to the window moments; the backward filters those three maps the same way
// (the window is symmetric, so the adjoint of the filter is the filter) and adds the gradient
// into dL/dC.  Both kernels fetch the next channel's
// block into registers while the current one is filtered, so its global-load latency is hidden.
//
// Loss values never go through same-address atomics (thousands of blocks adding into one cache
// line serialise in the memory system): every block writes its partial sum, and one block adds
// the partials in a fixed order, which also makes the loss value reproducible.
#include "gsr_internal.h"

namespace gsr {

constexpr int kMaskTX = 64, kMaskTY = 16;    // 256 lanes x 4 rows
constexpr int kMaxErode = 8;
constexpr int kCountBlocks = 16;             // mask-count blocks per view
constexpr int kL1Blocks = 256;               // masked-L1 blocks per view (grid-stride inside)
constexpr int kSsimR = 5;                    // window radius (11 taps)
constexpr int kSsimK = 2 * kSsimR + 1;
constexpr int kSsimTX = 32, kSsimTY = 32;    // output tile: 256 lanes x 4 pixels (a column of 4)
constexpr int kSsimRPT = kSsimTY / 8;         // output rows per lane
constexpr int kSsimRX = kSsimTX + 2 * kSsimR, kSsimRY = kSsimTY + 2 * kSsimR;  // 42 x 42 staged
constexpr int kSsimN = kSsimRX * kSsimRY;
constexpr int kSsimJ = (kSsimN + 255) / 256;  // staged elements per lane
constexpr float kSsimC1 = 0.01f * 0.01f, kSsimC2 = 0.03f * 0.03f;

struct SsimTaps {
    float g[kSsimK];
};

// ---- Eq. 7: support mask and its erosion -----------------------------------------------------
// One 64 x 16 pixel tile per block; the tile plus an r-pixel frame of M_geo is staged in LDS and
// every pixel tests its disk.
__global__ __launch_bounds__(256) void k_support_mask(const float *__restrict__ T, int W, int H, float thr, int r,
                                                      uint8_t *__restrict__ mask) {
    __shared__ uint8_t s_geo[(kMaskTY + 2 * kMaxErode) * (kMaskTX + 2 * kMaxErode)];
    const int v = blockIdx.z;
    const int x0 = blockIdx.x * kMaskTX, y0 = blockIdx.y * kMaskTY;
    const int RW = kMaskTX + 2 * r, RH = kMaskTY + 2 * r;
    const float *Tv = T + (int64_t)v * W * H;
    for (int e = threadIdx.x; e < RW * RH; e += 256) {
        const int gx = x0 - r + e % RW, gy = y0 - r + e / RW;
        uint8_t g = 0;
        if (gx >= 0 && gx < W && gy >= 0 && gy < H) g = Tv[(int64_t)gy * W + gx] <= thr;
        s_geo[e] = g;
    }
    __syncthreads();
    const int lx = threadIdx.x % kMaskTX, x = x0 + lx;
    const int r2 = r * r;
    for (int ly = threadIdx.x / kMaskTX; ly < kMaskTY; ly += 256 / kMaskTX) {
        const int y = y0 + ly;
        if (x >= W || y >= H) continue;
        uint32_t all = 1;
        for (int dy = -r; dy <= r; dy++) {
            const uint8_t *row = s_geo + (ly + r + dy) * RW + lx + r;
            for (int dx = -r; dx <= r; dx++)
                if (dy * dy + dx * dx <= r2) all &= row[dx];
        }
        mask[(int64_t)v * W * H + (int64_t)y * W + x] = (uint8_t)all;
    }
}

// |M_int| per view: 16 blocks per view, one atomic each.  Mask bytes are 0 or 1, so the
// population count of a 32-bit word is the number of mask pixels in it.
__global__ __launch_bounds__(256) void k_mask_count(const uint8_t *__restrict__ mask, int64_t P,
                                                    uint32_t *__restrict__ count) {
    __shared__ uint32_t s_cnt[4];
    const int v = blockIdx.y;
    const uint8_t *m = mask + (int64_t)v * P;
    uint32_t c = 0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    if ((P & 15) == 0) {
        const uint4 *m4 = reinterpret_cast<const uint4 *>(m);
        for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < P / 16; e += stride) {
            const uint4 q = m4[e];
            c += __popc(q.x) + __popc(q.y) + __popc(q.z) + __popc(q.w);
        }
    } else {
        for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < P; e += stride) c += m[e];
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (lane_id() == 0) s_cnt[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
        if (t) atomicAdd(count + v, t);
    }
}

__device__ __forceinline__ float view_norm(const uint32_t *count, const uint8_t *mask, int64_t P, int64_t v) {
    if (!mask) return 1.0f / (float)P;
    const uint32_t c = count[v];
    return c ? 1.0f / (float)c : 0.0f;
}

// Block sum of a per-lane double (fixed order), returned to lane 0 of wave 0.
__device__ __forceinline__ double block_sum_d(double acc, double *s_red) {
    acc = wave_sum_d(acc);
    if (lane_id() == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    return (s_red[0] + s_red[1]) + (s_red[2] + s_red[3]);
}

// ---- Eq. 10 and 12: masked L1 colour and depth -----------------------------------------------
// grid (kL1Blocks, V); partial[v * kL1Blocks + b] = this block's share of the view's loss.
__global__ __launch_bounds__(256) void k_loss_masked(const float *__restrict__ rgb, const float *__restrict__ depth,
                                                     const float *__restrict__ trgb, const float *__restrict__ tdepth,
                                                     const int32_t *__restrict__ tidx, const uint8_t *__restrict__ mask,
                                                     const uint32_t *__restrict__ count, int64_t P, float lam_rgb,
                                                     float lam_d, float *__restrict__ grgb, float *__restrict__ gdepth,
                                                     double *__restrict__ partial) {
    __shared__ double s_red[4];
    const int64_t v = blockIdx.y;
    const int64_t slot = tidx ? (int64_t)tidx[v] : v;
    const float norm = view_norm(count, mask, P, v);
    const uint8_t *mv = mask ? mask + v * P : nullptr;
    const float *C = rgb + v * 3 * P, *Ct = trgb + slot * 3 * P;
    const float *D = depth ? depth + v * P : nullptr, *Dt = tdepth ? tdepth + slot * P : nullptr;
    float *gC = grgb + v * 3 * P, *gD = gdepth ? gdepth + v * P : nullptr;
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < P; p += (int64_t)gridDim.x * 256) {
        const float inv = (!mv || mv[p]) ? norm : 0.0f;
        const float gc = lam_rgb * inv;
        float l = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            const float d = C[ch * P + p] - Ct[ch * P + p];
            l += fabsf(d);
            gC[ch * P + p] = d > 0.f ? gc : (d < 0.f ? -gc : 0.f);
        }
        l *= lam_rgb;
        float gd = 0.f;
        if (Dt) {
            const float d = D[p] - Dt[p];
            l += lam_d * fabsf(d);
            gd = d > 0.f ? lam_d * inv : (d < 0.f ? -lam_d * inv : 0.f);
        }
        if (gD) gD[p] = gd;
        if (inv != 0.0f) acc += (double)l * (double)inv;
    }
    const double t = block_sum_d(acc, s_red);
    if (threadIdx.x == 0) partial[v * gridDim.x + blockIdx.x] = t;
}

// Staging positions of one lane inside the 42 x 42 block (the same for every channel).
struct SsimStage {
    int64_t off[kSsimJ];
    bool in[kSsimJ];
    __device__ SsimStage(int x0, int y0, int W, int H) {
#pragma unroll
        for (int j = 0; j < kSsimJ; j++) {
            const int e = threadIdx.x + 256 * j;
            const int gx = x0 - kSsimR + e % kSsimRX, gy = y0 - kSsimR + e / kSsimRX;
            in[j] = e < kSsimN && gx >= 0 && gx < W && gy >= 0 && gy < H;
            off[j] = in[j] ? (int64_t)gy * W + gx : 0;
        }
    }
};

// ---- Eq. 11: SSIM forward -------------------------------------------------------------------
// maps [V][3 channels][3][H][W] = d loss / d(window mean of x, of x^2, of x y), zero off the
// mask.  partial[block] = this block's share of lambda (1 - sum_M sum_c S / (3 |M|)).
__global__ __launch_bounds__(256) void k_ssim_fwd(const float *__restrict__ rgb, const float *__restrict__ trgb,
                                                  const int32_t *__restrict__ tidx, const uint8_t *__restrict__ mask,
                                                  const uint32_t *__restrict__ count, int W, int H, float lam,
                                                  SsimTaps taps, float *__restrict__ maps,
                                                  double *__restrict__ partial) {
    __shared__ __align__(16) float s_x[kSsimN];
    __shared__ __align__(16) float s_y[kSsimN];
    __shared__ __align__(16) float s_h[5][kSsimRY][kSsimTX];
    __shared__ double s_red[4];
    const int v = blockIdx.z;
    const int64_t P = (int64_t)W * H;
    const int64_t bid = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    const float norm = view_norm(count, mask, P, v);
    if (norm == 0.0f) {  // empty mask: no loss, maps unused
        if (threadIdx.x == 0) partial[bid] = 0.0;
        return;
    }
    const int64_t slot = tidx ? (int64_t)tidx[v] : v;
    const int x0 = blockIdx.x * kSsimTX, y0 = blockIdx.y * kSsimTY;
    const float scale = -lam * norm * (1.0f / 3.0f);  // d loss / d S at a mask pixel
    const uint8_t *mv = mask ? mask + v * P : nullptr;
    const SsimStage st(x0, y0, W, H);
    bool use[kSsimJ];
#pragma unroll
    for (int j = 0; j < kSsimJ; j++) use[j] = st.in[j] && (!mv || mv[st.off[j]]);
    float ra[kSsimJ], rb[kSsimJ];
    auto fetch = [&](int ch) {
        const float *X = rgb + (v * 3 + ch) * P, *Y = trgb + (slot * 3 + ch) * P;
#pragma unroll
        for (int j = 0; j < kSsimJ; j++) {
            const float a = X[st.off[j]], b = Y[st.off[j]];
            ra[j] = use[j] ? a : 0.f;
            rb[j] = use[j] ? b : 0.f;
        }
    };
    const int lx = threadIdx.x % kSsimTX, ly0 = kSsimRPT * (threadIdx.x / kSsimTX);  // rows ly0 .. + RPT - 1
    double acc = 0.0;
    fetch(0);
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
#pragma unroll
        for (int j = 0; j < kSsimJ; j++) {
            const int e = threadIdx.x + 256 * j;
            if (e < kSsimN) {
                s_x[e] = ra[j];
                s_y[e] = rb[j];
            }
        }
        __syncthreads();
        if (ch < 2) fetch(ch + 1);
        // horizontal pass: 42 rows x 16 column pairs; 12 staged values feed two outputs
        for (int it = threadIdx.x; it < kSsimRY * (kSsimTX / 2); it += 256) {
            const int rr = it / (kSsimTX / 2), c0 = 2 * (it % (kSsimTX / 2));
            const float2 *px = reinterpret_cast<const float2 *>(s_x + rr * kSsimRX + c0);
            const float2 *py = reinterpret_cast<const float2 *>(s_y + rr * kSsimRX + c0);
            float m0[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, m1[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            auto elem = [&](float a, float b, int k) {
                const float aa = a * a, bb = b * b, ab = a * b;
                if (k < kSsimK) {
                    const float g = taps.g[k];
                    m0[0] += g * a, m0[1] += g * b, m0[2] += g * aa, m0[3] += g * bb, m0[4] += g * ab;
                }
                if (k >= 1) {
                    const float g = taps.g[k - 1];
                    m1[0] += g * a, m1[1] += g * b, m1[2] += g * aa, m1[3] += g * bb, m1[4] += g * ab;
                }
            };
#pragma unroll
            for (int k2 = 0; k2 < (kSsimK + 1) / 2; k2++) {
                const float2 a = px[k2], b = py[k2];
                elem(a.x, b.x, 2 * k2);
                elem(a.y, b.y, 2 * k2 + 1);
            }
#pragma unroll
            for (int q = 0; q < 5; q++) *reinterpret_cast<float2 *>(&s_h[q][rr][c0]) = make_float2(m0[q], m1[q]);
        }
        __syncthreads();
        // vertical pass: the kSsimRPT rows of column lx share kSsimRPT + 10 horizontal sums
        float o[kSsimRPT][5];
#pragma unroll
        for (int i = 0; i < kSsimRPT; i++)
#pragma unroll
            for (int q = 0; q < 5; q++) o[i][q] = 0.f;
#pragma unroll
        for (int k = 0; k < kSsimK + kSsimRPT - 1; k++) {
#pragma unroll
            for (int q = 0; q < 5; q++) {
                const float h = s_h[q][ly0 + k][lx];
#pragma unroll
                for (int i = 0; i < kSsimRPT; i++)
                    if (k - i >= 0 && k - i < kSsimK) o[i][q] += taps.g[k - i] * h;
            }
        }
#pragma unroll
        for (int i = 0; i < kSsimRPT; i++) {
            const int x = x0 + lx, y = y0 + ly0 + i;
            if (x >= W || y >= H) continue;
            const int64_t p = (int64_t)y * W + x;
            const bool in = !mv || mv[p];
            const float mx = o[i][0], my = o[i][1];
            const float vx = o[i][2] - mx * mx, vy = o[i][3] - my * my, cxy = o[i][4] - mx * my;
            const float n1 = 2.f * mx * my + kSsimC1, d1 = mx * mx + my * my + kSsimC1;
            const float n2 = 2.f * cxy + kSsimC2, d2 = vx + vy + kSsimC2;
            const float rd1 = 1.f / d1, rd2 = 1.f / d2;
            const float lum = n1 * rd1, cs = n2 * rd2, S = lum * cs;
            float ga = 0.f, gb = 0.f, ge = 0.f;
            if (in) {
                acc += (double)S;
                const float dl = 2.f * (my - mx * lum) * rd1, dc = 2.f * (mx * cs - my) * rd2;
                ga = scale * (cs * dl + lum * dc);
                gb = scale * (-S * rd2);
                ge = scale * (2.f * lum * rd2);
            }
            float *mp = maps + ((int64_t)(v * 3 + ch) * 3) * P + p;
            mp[0] = ga;
            mp[P] = gb;
            mp[2 * P] = ge;
        }
    }
    double t = (double)scale * block_sum_d(acc, s_red);
    if (threadIdx.x == 0) {
        if (blockIdx.x == 0 && blockIdx.y == 0) t += (double)lam;
        partial[bid] = t;
    }
}

// ---- Eq. 11: SSIM backward ------------------------------------------------------------------
// dL/dX(q) = (w * a)(q) + 2 X(q) (w * b)(q) + Y(q) (w * e)(q) with X, Y the masked images, then
// dL/dC = M dL/dX, ADDED into grgb.
__global__ __launch_bounds__(256) void k_ssim_bwd(const float *__restrict__ rgb, const float *__restrict__ trgb,
                                                  const int32_t *__restrict__ tidx, const uint8_t *__restrict__ mask,
                                                  const uint32_t *__restrict__ count, int W, int H, SsimTaps taps,
                                                  const float *__restrict__ maps, float *__restrict__ grgb) {
    __shared__ __align__(16) float s_m[3][kSsimN];
    __shared__ __align__(16) float s_h[3][kSsimRY][kSsimTX];
    const int v = blockIdx.z;
    const int64_t P = (int64_t)W * H;
    if (view_norm(count, mask, P, v) == 0.0f) return;
    const int64_t slot = tidx ? (int64_t)tidx[v] : v;
    const int x0 = blockIdx.x * kSsimTX, y0 = blockIdx.y * kSsimTY;
    const uint8_t *mv = mask ? mask + v * P : nullptr;
    const SsimStage st(x0, y0, W, H);
    float ra[kSsimJ], rb[kSsimJ], rc[kSsimJ];
    auto fetch = [&](int ch) {
        const float *mp = maps + ((int64_t)(v * 3 + ch) * 3) * P;
#pragma unroll
        for (int j = 0; j < kSsimJ; j++) {
            const float a = mp[st.off[j]], b = mp[P + st.off[j]], c = mp[2 * P + st.off[j]];
            ra[j] = st.in[j] ? a : 0.f;
            rb[j] = st.in[j] ? b : 0.f;
            rc[j] = st.in[j] ? c : 0.f;
        }
    };
    const int lx = threadIdx.x % kSsimTX, ly0 = kSsimRPT * (threadIdx.x / kSsimTX);
    const int x = x0 + lx;
    bool out[kSsimRPT];
    int64_t pix[kSsimRPT];
#pragma unroll
    for (int i = 0; i < kSsimRPT; i++) {
        const int y = y0 + ly0 + i;
        out[i] = x < W && y < H;
        pix[i] = out[i] ? (int64_t)y * W + x : 0;
        out[i] = out[i] && (!mv || mv[pix[i]]);
    }
    fetch(0);
#pragma unroll
    for (int ch = 0; ch < 3; ch++) {
#pragma unroll
        for (int j = 0; j < kSsimJ; j++) {
            const int e = threadIdx.x + 256 * j;
            if (e < kSsimN) {
                s_m[0][e] = ra[j];
                s_m[1][e] = rb[j];
                s_m[2][e] = rc[j];
            }
        }
        __syncthreads();
        if (ch < 2) fetch(ch + 1);
        float X[kSsimRPT], Y[kSsimRPT], G[kSsimRPT];
        float *gC = grgb + (v * 3 + ch) * P;
#pragma unroll
        for (int i = 0; i < kSsimRPT; i++) {
            X[i] = out[i] ? rgb[(v * 3 + ch) * P + pix[i]] : 0.f;
            Y[i] = out[i] ? trgb[(slot * 3 + ch) * P + pix[i]] : 0.f;
            G[i] = out[i] ? gC[pix[i]] : 0.f;
        }
        for (int it = threadIdx.x; it < kSsimRY * (kSsimTX / 2); it += 256) {
            const int rr = it / (kSsimTX / 2), c0 = 2 * (it % (kSsimTX / 2));
            float h0[3] = {0.f, 0.f, 0.f}, h1[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int k2 = 0; k2 < (kSsimK + 1) / 2; k2++) {
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    const float2 m = *reinterpret_cast<const float2 *>(&s_m[q][rr * kSsimRX + c0 + 2 * k2]);
                    const int k = 2 * k2;
                    h0[q] += taps.g[k] * m.x;
                    if (k + 1 < kSsimK) h0[q] += taps.g[k + 1] * m.y;
                    if (k >= 1) h1[q] += taps.g[k - 1] * m.x;
                    h1[q] += taps.g[k] * m.y;
                }
            }
#pragma unroll
            for (int q = 0; q < 3; q++) *reinterpret_cast<float2 *>(&s_h[q][rr][c0]) = make_float2(h0[q], h1[q]);
        }
        __syncthreads();
        float o[kSsimRPT][3];
#pragma unroll
        for (int i = 0; i < kSsimRPT; i++) o[i][0] = o[i][1] = o[i][2] = 0.f;
#pragma unroll
        for (int k = 0; k < kSsimK + kSsimRPT - 1; k++) {
#pragma unroll
            for (int q = 0; q < 3; q++) {
                const float h = s_h[q][ly0 + k][lx];
#pragma unroll
                for (int i = 0; i < kSsimRPT; i++)
                    if (k - i >= 0 && k - i < kSsimK) o[i][q] += taps.g[k - i] * h;
            }
        }
#pragma unroll
        for (int i = 0; i < kSsimRPT; i++)
            if (out[i]) gC[pix[i]] = G[i] + (o[i][0] + 2.f * X[i] * o[i][1] + Y[i] * o[i][2]);
    }
}

// loss += sum of n partials, in a fixed order (one block of 1024 lanes, four loads in flight).
__global__ __launch_bounds__(1024) void k_loss_reduce(const double *__restrict__ partial, int64_t n,
                                                      double *__restrict__ loss) {
    __shared__ double s_red[16];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int64_t e = threadIdx.x;
    for (; e + 3 * 1024 < n; e += 4 * 1024) {
        a0 += partial[e];
        a1 += partial[e + 1024];
        a2 += partial[e + 2048];
        a3 += partial[e + 3072];
    }
    for (; e < n; e += 1024) a0 += partial[e];
    double acc = wave_sum_d((a0 + a1) + (a2 + a3));
    if (lane_id() == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; w++) t += s_red[w];
        *loss += t;
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

int64_t ssim_blocks(int V, const gsr_raster *r) {
    return ceil_div(r->width, kSsimTX) * ceil_div(r->height, kSsimTY) * (int64_t)V;
}

}  // namespace gsr

using namespace gsr;

extern "C" gsr_status gsr_fill_u32_launch(void *, uint32_t, int64_t, hipStream_t);

// Workspace: [SSIM derivative maps: V * 9 * P floats][partials: V * kL1Blocks + ssim blocks doubles]
extern "C" size_t gsr_loss_ws_bytes(int V, const gsr_raster *r) {
    return align256((size_t)V * 9 * (size_t)r->width * r->height * sizeof(float)) +
           align256((size_t)(V * kL1Blocks + ssim_blocks(V, r)) * sizeof(double));
}

extern "C" gsr_status gsr_support_mask_launch(const float *T, int V, const gsr_raster *r, float tau, int rad,
                                              uint8_t *mask, uint32_t *count, hipStream_t st) {
    gsr_status s = gsr_fill_u32_launch(count, 0u, V, st);
    if (s != GSR_OK) return s;
    const float thr = 1.0f - tau;
    dim3 grid((unsigned)ceil_div(r->width, kMaskTX), (unsigned)ceil_div(r->height, kMaskTY), (unsigned)V);
    k_support_mask<<<grid, 256, 0, st>>>(T, r->width, r->height, thr, rad, mask);
    k_mask_count<<<dim3(kCountBlocks, V), 256, 0, st>>>(mask, (int64_t)r->width * r->height, count);
    return last_launch();
}

extern "C" gsr_status gsr_loss_launch(const float *rgb, const float *depth, const float *trgb, const float *tdepth,
                                      const int32_t *tidx, int V, const gsr_raster *r, const uint8_t *mask,
                                      const uint32_t *count, float lam_rgb, float lam_ssim, float lam_d, double *loss,
                                      float *grgb, float *gdepth, void *ws, hipStream_t st) {
    const int64_t P = (int64_t)r->width * r->height;
    float *maps = static_cast<float *>(ws);
    double *partial = reinterpret_cast<double *>(static_cast<char *>(ws) + align256((size_t)V * 9 * P * sizeof(float)));
    k_loss_masked<<<dim3(kL1Blocks, V), 256, 0, st>>>(rgb, depth, trgb, tdepth, tidx, mask, count, P, lam_rgb, lam_d,
                                                      grgb, gdepth, partial);
    int64_t n_part = (int64_t)V * kL1Blocks;
    if (lam_ssim != 0.0f) {
        SsimTaps taps;
        double g[kSsimK], sum = 0.0;
        for (int k = -kSsimR; k <= kSsimR; k++) sum += g[k + kSsimR] = exp(-(double)(k * k) / (2.0 * 1.5 * 1.5));
        for (int k = 0; k < kSsimK; k++) taps.g[k] = (float)(g[k] / sum);
        dim3 grid((unsigned)ceil_div(r->width, kSsimTX), (unsigned)ceil_div(r->height, kSsimTY), (unsigned)V);
        k_ssim_fwd<<<grid, 256, 0, st>>>(rgb, trgb, tidx, mask, count, r->width, r->height, lam_ssim, taps, maps,
                                         partial + n_part);
        k_ssim_bwd<<<grid, 256, 0, st>>>(rgb, trgb, tidx, mask, count, r->width, r->height, taps, maps, grgb);
        n_part += ssim_blocks(V, r);
    }
    k_loss_reduce<<<1, 1024, 0, st>>>(partial, n_part, loss);
    return last_launch();
}
