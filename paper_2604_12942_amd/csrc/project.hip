// EWA projection of 3-D Gaussians into pinhole views, and its exact backward with the camera-pose
// gradient.  One thread per Gaussian walks every view, so the per-Gaussian parameters (up to 236
// bytes at SH degree 3) are read from HBM once per step instead of once per view, and the
// parameter gradients are accumulated over views in registers (no atomics, no re-reads).
// The arithmetic is double precision: the stage is bound by HBM traffic, and FP64 keeps the
// screen-space results within a rounding of the exact values of the float32 inputs.
#include "gsr_internal.h"

#include <mutex>

namespace gsr {

// Real spherical harmonics without Condon-Shortley phase, orthonormal, ordered (l, m = -l..l),
// as polynomials of the unit direction (x, y, z).
// Term k in float, with its polynomial gradient.  k is wave-uniform and the callers loop over it
// without unrolling, so one term's three coefficients (two terms' in the pipelined backward) are
// live at a time: unrolling the basis would keep every coefficient load in flight and cap
// occupancy.
__device__ __forceinline__ float sh_term(int k, float x, float y, float z, float &gx, float &gy, float &gz) {
    constexpr float a = 0.4886025119029199f;
    constexpr float b = 1.0925484305920792f, c = 0.31539156525252005f, d = 0.5462742152960396f;
    constexpr float e = 0.5900435899266435f, f = 2.890611442640554f, g = 0.4570457994644658f;
    constexpr float h = 0.3731763325901154f, m = 1.445305721320277f;
    gx = gy = gz = 0.f;
    switch (k) {
        case 0: return 0.28209479177387814f;
        case 1: gy = a; return a * y;
        case 2: gz = a; return a * z;
        case 3: gx = a; return a * x;
        case 4: gx = b * y; gy = b * x; return b * x * y;
        case 5: gy = b * z; gz = b * y; return b * y * z;
        case 6: gz = 6.0f * c * z; return c * (3.0f * z * z - 1.0f);
        case 7: gx = b * z; gz = b * x; return b * x * z;
        case 8: gx = 2.0f * d * x; gy = -2.0f * d * y; return d * (x * x - y * y);
        case 9: gx = 6.0f * e * x * y; gy = 3.0f * e * (x * x - y * y); return e * y * (3.0f * x * x - y * y);
        case 10: gx = f * y * z; gy = f * x * z; gz = f * x * y; return f * x * y * z;
        case 11: gy = g * (5.0f * z * z - 1.0f); gz = 10.0f * g * y * z; return g * y * (5.0f * z * z - 1.0f);
        case 12: gz = h * (15.0f * z * z - 3.0f); return h * z * (5.0f * z * z - 3.0f);
        case 13: gx = g * (5.0f * z * z - 1.0f); gz = 10.0f * g * x * z; return g * x * (5.0f * z * z - 1.0f);
        case 14:
            gx = 2.0f * m * x * z; gy = -2.0f * m * y * z; gz = m * (x * x - y * y);
            return m * z * (x * x - y * y);
        default:
            gx = 3.0f * e * (x * x - y * y); gy = -6.0f * e * x * y;
            return e * x * (x * x - 3.0f * y * y);
    }
}

// pre-clamp colour 1/2 + sum_k Y_k(d) h_k, coefficients read from the component-major array
template <int K>
__device__ __forceinline__ void sh_colour(float x, float y, float z, const float *__restrict__ sh, int64_t n,
                                          int64_t i, float pre[3]) {
#pragma unroll 1
    for (int k = 0; k < K; k++) {
        float gx, gy, gz;
        const float Yk = sh_term(k, x, y, z, gx, gy, gz);
        pre[0] = __builtin_fmaf(Yk, sh[(3 * k + 0) * n + i], pre[0]);
        pre[1] = __builtin_fmaf(Yk, sh[(3 * k + 1) * n + i], pre[1]);
        pre[2] = __builtin_fmaf(Yk, sh[(3 * k + 2) * n + i], pre[2]);
    }
}

// the same sum fully unrolled: the forward projection keeps every coefficient load in flight.
// That costs registers (two waves per SIMD at degree 3), but a pipelined loop at four waves per
// SIMD was measured 25 % slower: the stage streams parameters, and loads in flight matter more.
template <int K, int k = 0>
__device__ __forceinline__ void sh_colour_unrolled(float x, float y, float z, const float *__restrict__ sh, int64_t n,
                                                   int64_t i, float pre[3]) {
    if constexpr (k < K) {
        float gx, gy, gz;
        const float Yk = sh_term(k, x, y, z, gx, gy, gz);
        pre[0] = __builtin_fmaf(Yk, sh[(3 * k + 0) * n + i], pre[0]);
        pre[1] = __builtin_fmaf(Yk, sh[(3 * k + 1) * n + i], pre[1]);
        pre[2] = __builtin_fmaf(Yk, sh[(3 * k + 2) * n + i], pre[2]);
        sh_colour_unrolled<K, k + 1>(x, y, z, sh, n, i, pre);
    }
}

// backward of the colour: gh[k][ch] += gcol[ch] Y_k, gdir += (sum_ch gcol[ch] h_k,ch) grad Y_k.
// Software-pipelined: the next term's three coefficients are loaded while the current term is
// worked, so the walk does not wait out one memory round trip per term.
template <int K>
__device__ __forceinline__ void sh_colour_bwd(float x, float y, float z, const float *__restrict__ sh, int64_t n,
                                              int64_t i, const float gcol[3], float *gh, int stride, float gdir[3]) {
    float h0 = sh[i], h1 = sh[n + i], h2 = sh[2 * n + i];
#pragma unroll 1
    for (int k = 0; k < K; k++) {
        float n0 = 0.f, n1 = 0.f, n2 = 0.f;
        if (k + 1 < K) {
            n0 = sh[(3 * k + 3) * n + i];
            n1 = sh[(3 * k + 4) * n + i];
            n2 = sh[(3 * k + 5) * n + i];
        }
        float gx, gy, gz;
        const float Yk = sh_term(k, x, y, z, gx, gy, gz);
        const float hk[3] = {h0, h1, h2};
        float sk = 0.f;
#pragma unroll
        for (int ch = 0; ch < 3; ch++) {
            float &acc = gh[(3 * k + ch) * stride];
            acc = __builtin_fmaf(gcol[ch], Yk, acc);
            sk = __builtin_fmaf(gcol[ch], hk[ch], sk);
        }
        gdir[0] = __builtin_fmaf(sk, gx, gdir[0]);
        gdir[1] = __builtin_fmaf(sk, gy, gdir[1]);
        gdir[2] = __builtin_fmaf(sk, gz, gdir[2]);
        h0 = n0;
        h1 = n1;
        h2 = n2;
    }
}

// Rotation of a unit quaternion (w, v): R = (w^2 - |v|^2) I + 2 v v^T + 2 w [v]_x.
__device__ __forceinline__ void quat_rot(double w, double x, double y, double z, double R[3][3]) {
    const double s = w * w - (x * x + y * y + z * z);
    const double v[3] = {x, y, z};
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) R[a][b] = (a == b ? s : 0.0) + 2.0 * v[a] * v[b];
    R[0][1] -= 2.0 * w * z; R[1][0] += 2.0 * w * z;
    R[0][2] += 2.0 * w * y; R[2][0] -= 2.0 * w * y;
    R[1][2] -= 2.0 * w * x; R[2][1] += 2.0 * w * x;
}

struct Cam {
    double R[3][3], t[3], fx, fy, cx, cy, znear, C[3];
};

__device__ __forceinline__ void load_cam(const gsr_camera &c, Cam &k) {
    for (int a = 0; a < 3; a++) {
        for (int b = 0; b < 3; b++) k.R[a][b] = (double)c.R[3 * a + b];
        k.t[a] = (double)c.t[a];
    }
    k.fx = c.fx; k.fy = c.fy; k.cx = c.cx; k.cy = c.cy; k.znear = c.z_near;
    for (int a = 0; a < 3; a++) k.C[a] = -(k.R[0][a] * k.t[0] + k.R[1][a] * k.t[1] + k.R[2][a] * k.t[2]);
}

// symmetric 3x3: xx, xy, xz, yy, yz, zz
struct Sym3 {
    double xx, xy, xz, yy, yz, zz;
};

__device__ __forceinline__ double sym_at(const Sym3 &S, int a, int b) {
    const int k = a < b ? a * 3 + b : b * 3 + a;  // 0 1 2 / 4 5 / 8
    switch (k) {
        case 0: return S.xx;
        case 1: return S.xy;
        case 2: return S.xz;
        case 4: return S.yy;
        case 5: return S.yz;
        default: return S.zz;
    }
}

// R S R^T for a symmetric S
__device__ __forceinline__ Sym3 rot_sym(const double R[3][3], const Sym3 &S) {
    double RS[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            RS[a][b] = R[a][0] * sym_at(S, 0, b) + R[a][1] * sym_at(S, 1, b) + R[a][2] * sym_at(S, 2, b);
    Sym3 o;
    o.xx = RS[0][0] * R[0][0] + RS[0][1] * R[0][1] + RS[0][2] * R[0][2];
    o.xy = RS[0][0] * R[1][0] + RS[0][1] * R[1][1] + RS[0][2] * R[1][2];
    o.xz = RS[0][0] * R[2][0] + RS[0][1] * R[2][1] + RS[0][2] * R[2][2];
    o.yy = RS[1][0] * R[1][0] + RS[1][1] * R[1][1] + RS[1][2] * R[1][2];
    o.yz = RS[1][0] * R[2][0] + RS[1][1] * R[2][1] + RS[1][2] * R[2][2];
    o.zz = RS[2][0] * R[2][0] + RS[2][1] * R[2][1] + RS[2][2] * R[2][2];
    return o;
}

// R^T S R for a symmetric S
__device__ __forceinline__ Sym3 rot_sym_t(const double R[3][3], const Sym3 &S) {
    double Rt[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) Rt[a][b] = R[b][a];
    return rot_sym(Rt, S);
}

// Everything the forward and backward share for one (view, Gaussian).
struct ViewGeom {
    double p[3];        // camera-frame mean
    Sym3 Sc;            // camera-frame covariance
    double j00, j02, j11, j12, tx, ty;
    bool clx, cly;
    double a, b, c;     // Sigma' = [[a, b], [b, c]]
    double det;
    double u, v;
    double dir[3], dist;
};

__device__ __forceinline__ bool view_geom(const double mu[3], const Sym3 &Sig, const Cam &k, int W, int H,
                                          ViewGeom &G) {
    for (int a = 0; a < 3; a++) G.p[a] = k.R[a][0] * mu[0] + k.R[a][1] * mu[1] + k.R[a][2] * mu[2] + k.t[a];
    const double z = G.p[2];
    if (!(z > k.znear)) return false;
    G.Sc = rot_sym(k.R, Sig);
    const double limx = GSR_GUARD * W / (2.0 * k.fx), limy = GSR_GUARD * H / (2.0 * k.fy);
    const double rx = G.p[0] / z, ry = G.p[1] / z;
    G.clx = fabs(rx) > limx;
    G.cly = fabs(ry) > limy;
    G.tx = G.clx ? copysign(limx, rx) : rx;
    G.ty = G.cly ? copysign(limy, ry) : ry;
    const double iz = 1.0 / z;
    G.j00 = k.fx * iz; G.j02 = -k.fx * G.tx * iz;
    G.j11 = k.fy * iz; G.j12 = -k.fy * G.ty * iz;
    // Sigma' = J Sc J^T + 0.3 I with J = [[j00, 0, j02], [0, j11, j12]]
    const Sym3 &S = G.Sc;
    G.a = G.j00 * (G.j00 * S.xx + G.j02 * S.xz) + G.j02 * (G.j00 * S.xz + G.j02 * S.zz) + GSR_LOWPASS;
    G.b = G.j00 * (G.j11 * S.xy + G.j12 * S.xz) + G.j02 * (G.j11 * S.yz + G.j12 * S.zz);
    G.c = G.j11 * (G.j11 * S.yy + G.j12 * S.yz) + G.j12 * (G.j11 * S.yz + G.j12 * S.zz) + GSR_LOWPASS;
    G.det = G.a * G.c - G.b * G.b;
    G.u = k.fx * G.p[0] * iz + k.cx;
    G.v = k.fy * G.p[1] * iz + k.cy;
    double d[3] = {mu[0] - k.C[0], mu[1] - k.C[1], mu[2] - k.C[2]};
    G.dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double idist = 1.0 / G.dist;
    for (int a = 0; a < 3; a++) G.dir[a] = d[a] * idist;
    return true;
}

// unit quaternion and the norm of the stored one
__device__ __forceinline__ void unit_quat(const float qf[4], double qn[4], double &qnorm) {
    double q[4];
    for (int a = 0; a < 4; a++) q[a] = qf[a];
    qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int a = 0; a < 4; a++) qn[a] = q[a] / qnorm;
}

__device__ __forceinline__ void load_rotation_scale(const gsr_gaussians &g, int64_t i, float qf[4], float lsf[3]) {
    const int64_t n = g.n;
    for (int a = 0; a < 4; a++) qf[a] = g.quats[a * n + i];
    for (int a = 0; a < 3; a++) lsf[a] = g.log_scales[a * n + i];
}

// Sigma = Rq S S^T Rq^T from the stored quaternion and log-scales
__device__ __forceinline__ Sym3 sigma_of(const float qf[4], const float lsf[3]) {
    double qn[4], qnorm, Rq[3][3], s2[3];
    unit_quat(qf, qn, qnorm);
    quat_rot(qn[0], qn[1], qn[2], qn[3], Rq);
    for (int a = 0; a < 3; a++) {
        const double sa = exp((double)lsf[a]);
        s2[a] = sa * sa;
    }
    Sym3 S;
    S.xx = Rq[0][0] * Rq[0][0] * s2[0] + Rq[0][1] * Rq[0][1] * s2[1] + Rq[0][2] * Rq[0][2] * s2[2];
    S.xy = Rq[0][0] * Rq[1][0] * s2[0] + Rq[0][1] * Rq[1][1] * s2[1] + Rq[0][2] * Rq[1][2] * s2[2];
    S.xz = Rq[0][0] * Rq[2][0] * s2[0] + Rq[0][1] * Rq[2][1] * s2[1] + Rq[0][2] * Rq[2][2] * s2[2];
    S.yy = Rq[1][0] * Rq[1][0] * s2[0] + Rq[1][1] * Rq[1][1] * s2[1] + Rq[1][2] * Rq[1][2] * s2[2];
    S.yz = Rq[1][0] * Rq[2][0] * s2[0] + Rq[1][1] * Rq[2][1] * s2[1] + Rq[1][2] * Rq[2][2] * s2[2];
    S.zz = Rq[2][0] * Rq[2][0] * s2[0] + Rq[2][1] * Rq[2][1] * s2[1] + Rq[2][2] * Rq[2][2] * s2[2];
    return S;
}

__device__ __forceinline__ Sym3 gaussian_sigma(const gsr_gaussians &g, int64_t i) {
    float qf[4], lsf[3];
    load_rotation_scale(g, i, qf, lsf);
    return sigma_of(qf, lsf);
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project(gsr_gaussians g, const gsr_camera *__restrict__ cams, int V, int W,
                                                 int H, int tw, int th, gsr_splat *__restrict__ splats,
                                                 uint32_t *__restrict__ info) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int64_t n = g.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t VN = (int64_t)V * n;
    const double mu[3] = {g.means[i], g.means[n + i], g.means[2 * n + i]};
    const Sym3 Sig = gaussian_sigma(g, i);
    const double o = 1.0 / (1.0 + exp(-(double)g.opacity_logits[i]));
#pragma unroll 1
    for (int vi = 0; vi < V; vi++) {
        // keep the SH coefficients out of registers across views: they are re-read (cached) per view
        __asm__ __volatile__("" ::: "memory");
        Cam k;
        load_cam(cams[vi], k);
        const int64_t gid = vi * n + i;
        ViewGeom G;
        uint32_t ntiles = 0, zbits = 0, r0 = 0, r1 = 0;
        double2 rec0 = make_double2(0, 0);
        float4 rec1 = make_float4(0, 0, 0, 0), rec2 = make_float4(0, 0, 0, 0);
        if (view_geom(mu, Sig, k, W, H, G) && 255.0 * o >= 1.0) {
            // footprint: D^T Q D <= r2, bounding box half-extents sqrt(r2 a), sqrt(r2 c)
            const double r2 = 2.0 * log(255.0 * o);
            const double ex = sqrt(r2 * G.a), ey = sqrt(r2 * G.c);
            double fx0 = floor(G.u - ex - 0.5) - 1.0, fx1 = ceil(G.u + ex - 0.5) + 1.0;
            double fy0 = floor(G.v - ey - 0.5) - 1.0, fy1 = ceil(G.v + ey - 0.5) + 1.0;
            fx0 = fmax(fx0, 0.0); fy0 = fmax(fy0, 0.0);
            fx1 = fmin(fx1, (double)(W - 1)); fy1 = fmin(fy1, (double)(H - 1));
            if (fx0 <= fx1 && fy0 <= fy1 && G.det > 0.0) {  // NaNs fail these tests too
                const int x0 = (int)fx0, x1 = (int)fx1, y0 = (int)fy0, y1 = (int)fy1;
                const uint32_t tx0 = x0 / tw, tx1 = x1 / tw, ty0 = y0 / th, ty1 = y1 / th;
                ntiles = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
                r0 = tx0 | (ty0 << 16);
                r1 = tx1 | (ty1 << 16);
                const float zf = (float)G.p[2];
                zbits = __float_as_uint(zf);
                // colour in the viewing direction
                float col[3] = {0.5f, 0.5f, 0.5f};
                sh_colour_unrolled<K>((float)G.dir[0], (float)G.dir[1], (float)G.dir[2], g.sh, n, i, col);
                // Cholesky factor of kappa Q, Q = [[c, -b], [-b, a]] / det:
                // l11 = sqrt(kappa c / det), l21 = -kappa b / (det l11), l22 = sqrt(kappa / c)
                const double qa = GSR_KAPPA * G.c / G.det, qb = -GSR_KAPPA * G.b / G.det;
                const double l11 = sqrt(qa);
                rec0 = make_double2(G.u, G.v);
                rec1 = make_float4((float)l11, (float)(qb / l11), (float)sqrt(GSR_KAPPA / G.c), (float)o);
                rec2 = make_float4(zf, fmaxf(col[0], 0.f), fmaxf(col[1], 0.f), fmaxf(col[2], 0.f));
            }
        }
        // only visible pairs are ever read back: skip the record writes of the others
        info[gid] = ntiles;
        if (ntiles) {
            *reinterpret_cast<double2 *>(splats + gid) = rec0;
            float4 *dstf = reinterpret_cast<float4 *>(splats + gid) + 1;
            dstf[0] = rec1;
            dstf[1] = rec2;
            info[VN + gid] = zbits;
            info[2 * VN + gid] = r0;
            info[3 * VN + gid] = r1;
        }
    }
}

// ---------------------------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------------------------
// Sum over the wave in float (DPP row shifts, then row broadcasts): the total lands in lane 63.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add(float v) {
    return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xf, false));
}
__device__ __forceinline__ float wave_total_f(float v) {
    v = dpp_add<0x111, 0xf>(v);  // row_shr:1
    v = dpp_add<0x112, 0xf>(v);  // row_shr:2
    v = dpp_add<0x114, 0xf>(v);  // row_shr:4
    v = dpp_add<0x118, 0xf>(v);  // row_shr:8
    v = dpp_add<0x142, 0xa>(v);  // row_bcast:15
    v = dpp_add<0x143, 0xc>(v);  // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// In-place Adam on the first cnt (at most N) elements of one Gaussian's row of a parameter group,
// element k at base + k * stride, with the same float expression as the standalone optimiser
// kernel. The three arrays never overlap: every load is issued before any store, so the elements
// do not each wait out a separate memory round trip.
template <int N>
__device__ __forceinline__ void adam_batch(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                                           int64_t base, int64_t stride, int cnt, const float *g, const float *lr,
                                           float b1, float b2, float eps, float bc1, float bc2) {
    float pm[N], mv[N], vv[N];
#pragma unroll
    for (int k = 0; k < N; k++) {
        if (k >= cnt) break;
        pm[k] = p[base + k * stride];
        mv[k] = m[base + k * stride];
        vv[k] = v[base + k * stride];
    }
#pragma unroll
    for (int k = 0; k < N; k++) {
        if (k >= cnt) break;
        const float mm = b1 * mv[k] + (1.0f - b1) * g[k];
        const float v2 = b2 * vv[k] + (1.0f - b2) * g[k] * g[k];
        m[base + k * stride] = mm;
        v[base + k * stride] = v2;
        p[base + k * stride] = pm[k] - lr[k] * (mm / bc1) / (sqrtf(v2 / bc2) + eps);
    }
}

struct FusedAdam {
    gsr_param_grads m, v;
    float lr[6];
    float b1, b2, eps;
    const int32_t *step;
};

// Chain rule from the screen-space gradients (per pair, dsplat) to the parameters and the
// per-view pose.  A Gaussian that no view rendered costs V 4-byte reads of tile_info and nothing
// else.  FUSED:
// instead of accumulating gradients, visible Gaussians of unfrozen segments take their sparse
// Adam step directly from the register-held gradient (no gradient buffer round trip).  The SH
// coefficient gradients accumulate across views in LDS ([coefficient][thread], conflict-free).
template <int DEG, bool FUSED>
__global__ __launch_bounds__(256) void k_project_bwd(gsr_gaussians g, const gsr_camera *__restrict__ cams, int V,
                                                     int W, int H, const gsr_splat *__restrict__ splats,
                                                     const float *__restrict__ dsplat,
                                                     gsr_param_grads out, double *__restrict__ pose_part,
                                                     const uint32_t *__restrict__ tile_info,
                                                     const int32_t *__restrict__ seg, int32_t min_seg,
                                                     uint8_t *__restrict__ row_mask, FusedAdam adam,
                                                     const uint32_t *__restrict__ vlist,
                                                     const uint32_t *__restrict__ vcount) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    __shared__ float s_gh[3 * K][256];
    const int64_t n = g.n;
    // thread -> Gaussian: directly, or through the compacted list of visible Gaussians
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t cnt = vlist ? (int64_t)*vcount : n;
    if ((int64_t)blockIdx.x * blockDim.x >= cnt) {
        // past the end of the (visible) list: the pose reduction reads only the partials of
        // the blocks below this one
        return;
    }
    const bool live = t < cnt;
    const int64_t i = live ? (vlist ? (int64_t)vlist[t] : t) : 0;
    // the views that rendered this Gaussian (bit vi; at most 32 views are tracked this way, the
    // rest are read where they are needed)
    uint32_t vmask = 0;
    bool anyvis = false;
    if (live)
        for (int vi = 0; vi < V; vi++) {
            const bool vis = tile_info[(int64_t)vi * n + i] > 0;
            anyvis |= vis;
            if (vi < 32) vmask |= (vis ? 1u : 0u) << vi;
        }
    float *gh = &s_gh[0][threadIdx.x];
#pragma unroll
    for (int e = 0; e < 3 * K; e++) gh[e * 256] = 0.f;
    double mu[3] = {0, 0, 0};
    Sym3 Sig{1, 0, 0, 1, 0, 1};
    double o = 0;
    // the stored rotation and scales, kept for the chain rule after the view loop
    float qf[4] = {1.f, 0.f, 0.f, 0.f}, lsf[3] = {0.f, 0.f, 0.f};
    if (anyvis) {
        for (int a = 0; a < 3; a++) mu[a] = g.means[a * n + i];
        load_rotation_scale(g, i, qf, lsf);
        Sig = sigma_of(qf, lsf);
        o = 1.0 / (1.0 + exp(-(double)g.opacity_logits[i]));
    }
    Sym3 gSig{0, 0, 0, 0, 0, 0};
    double gmu[3] = {0, 0, 0}, gop = 0;
    bool touched = false, visible = false;

#pragma unroll 1
    for (int vi = 0; vi < V; vi++) {
        __asm__ __volatile__("" ::: "memory");
        double pose[6] = {0, 0, 0, 0, 0, 0};
        float gs[10];
        float4 rgbz = make_float4(0.f, 0.f, 0.f, 0.f);
        bool any = false;
        if (anyvis) {
            // only rendered pairs hold gradients (summed per pair beforehand)
            const bool vis = vi < 32 ? ((vmask >> vi) & 1u) != 0 : tile_info[(int64_t)vi * n + i] > 0;
            visible |= vis;
#pragma unroll
            for (int e = 0; e < 10; e++) gs[e] = 0.f;
            if (vis) {
                const float2 *s2 = reinterpret_cast<const float2 *>(dsplat + ((int64_t)vi * n + i) * GSR_SPLAT_GRAD_FLOATS);
                // the splat's clamped colour, loaded with the gradients (one round trip per view)
                rgbz = *(reinterpret_cast<const float4 *>(splats + (int64_t)vi * n + i) + 2);
#pragma unroll
                for (int e = 0; e < 5; e++) {
                    const float2 q = s2[e];
                    gs[2 * e] = q.x;
                    gs[2 * e + 1] = q.y;
                }
#pragma unroll
                for (int e = 0; e < 10; e++) any |= gs[e] != 0.f;
            }
        }
        Cam k;
        load_cam(cams[vi], k);
        ViewGeom G;
        if (any && view_geom(mu, Sig, k, W, H, G)) {
            touched = true;
            const double x = G.p[0], y = G.p[1], z = G.p[2], iz = 1.0 / z;
            // conic Q = [[c, -b], [-b, a]] / det
            const double idet = 1.0 / G.det;
            const double Qa = G.c * idet, Qb = -G.b * idet, Qc = G.a * idet;
            // dL/dSigma' = -Q dL/dQ Q with the symmetric dL/dQ = [[ga, gb/2], [gb/2, gc]]
            const double ga = gs[2], gb = 0.5 * gs[3], gc = gs[4];
            const double m00 = Qa * ga + Qb * gb, m01 = Qa * gb + Qb * gc;
            const double m10 = Qb * ga + Qc * gb, m11 = Qb * gb + Qc * gc;
            const double S00 = -(m00 * Qa + m01 * Qb), S01 = -(m00 * Qb + m01 * Qc);
            const double S11 = -(m10 * Qb + m11 * Qc);
            // J rows: J0 = (j00, 0, j02), J1 = (0, j11, j12); dL/dSc = J^T dL/dSigma' J
            const double J0[3] = {G.j00, 0.0, G.j02}, J1[3] = {0.0, G.j11, G.j12};
            Sym3 gSc;
            gSc.xx = J0[0] * (S00 * J0[0] + S01 * J1[0]) + J1[0] * (S01 * J0[0] + S11 * J1[0]);
            gSc.xy = J0[0] * (S00 * J0[1] + S01 * J1[1]) + J1[0] * (S01 * J0[1] + S11 * J1[1]);
            gSc.xz = J0[0] * (S00 * J0[2] + S01 * J1[2]) + J1[0] * (S01 * J0[2] + S11 * J1[2]);
            gSc.yy = J0[1] * (S00 * J0[1] + S01 * J1[1]) + J1[1] * (S01 * J0[1] + S11 * J1[1]);
            gSc.yz = J0[1] * (S00 * J0[2] + S01 * J1[2]) + J1[1] * (S01 * J0[2] + S11 * J1[2]);
            gSc.zz = J0[2] * (S00 * J0[2] + S01 * J1[2]) + J1[2] * (S01 * J0[2] + S11 * J1[2]);
            // dL/dJ = 2 dL/dSigma' J Sc (rows 0 and 1)
            const Sym3 &Sc = G.Sc;
            const double JS0x = J0[0] * Sc.xx + J0[2] * Sc.xz, JS0y = J0[0] * Sc.xy + J0[2] * Sc.yz;
            const double JS0z = J0[0] * Sc.xz + J0[2] * Sc.zz;
            const double JS1x = J1[1] * Sc.xy + J1[2] * Sc.xz, JS1y = J1[1] * Sc.yy + J1[2] * Sc.yz;
            const double JS1z = J1[1] * Sc.yz + J1[2] * Sc.zz;
            const double gJ00 = 2.0 * (S00 * JS0x + S01 * JS1x);
            const double gJ02 = 2.0 * (S00 * JS0z + S01 * JS1z);
            const double gJ11 = 2.0 * (S01 * JS0y + S11 * JS1y);
            const double gJ12 = 2.0 * (S01 * JS0z + S11 * JS1z);
            // camera-frame point
            double gp[3];
            gp[0] = gs[0] * k.fx * iz;
            gp[1] = gs[1] * k.fy * iz;
            gp[2] = (double)gs[9] - gs[0] * k.fx * x * iz * iz - gs[1] * k.fy * y * iz * iz -
                    gJ00 * k.fx * iz * iz - gJ11 * k.fy * iz * iz;
            if (G.clx) {
                gp[2] += gJ02 * k.fx * G.tx * iz * iz;
            } else {
                gp[0] -= gJ02 * k.fx * iz * iz;
                gp[2] += gJ02 * 2.0 * k.fx * x * iz * iz * iz;
            }
            if (G.cly) {
                gp[2] += gJ12 * k.fy * G.ty * iz * iz;
            } else {
                gp[1] -= gJ12 * k.fy * iz * iz;
                gp[2] += gJ12 * 2.0 * k.fy * y * iz * iz * iz;
            }
            // world covariance: dL/dSigma += R^T dL/dSc R
            const Sym3 gw = rot_sym_t(k.R, gSc);
            gSig.xx += gw.xx; gSig.xy += gw.xy; gSig.xz += gw.xz;
            gSig.yy += gw.yy; gSig.yz += gw.yz; gSig.zz += gw.zz;
            // pose, rotation part through Sc: <dL/dSc, [e]x Sc - Sc [e]x> = 2 tr([e]x Sc dL/dSc)
            double A[3][3];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    A[a][b] = sym_at(Sc, a, 0) * sym_at(gSc, 0, b) + sym_at(Sc, a, 1) * sym_at(gSc, 1, b) +
                              sym_at(Sc, a, 2) * sym_at(gSc, 2, b);
            pose[3] += 2.0 * (A[1][2] - A[2][1]);
            pose[4] += 2.0 * (A[2][0] - A[0][2]);
            pose[5] += 2.0 * (A[0][1] - A[1][0]);
            // p = R mu + t
            for (int a = 0; a < 3; a++) gmu[a] += k.R[0][a] * gp[0] + k.R[1][a] * gp[1] + k.R[2][a] * gp[2];
            for (int a = 0; a < 3; a++) pose[a] += gp[a];
            pose[3] += y * gp[2] - z * gp[1];
            pose[4] += z * gp[0] - x * gp[2];
            pose[5] += x * gp[1] - y * gp[0];
            // colour: clamp at zero, SH coefficients, viewing direction.  The forward stored
            // max(0, pre-clamp colour) in the splat, so a zero channel is exactly a clamped one.
            const float dxf = (float)G.dir[0], dyf = (float)G.dir[1], dzf = (float)G.dir[2];
            float gcol[3], gdirf[3] = {0.f, 0.f, 0.f};
            gcol[0] = rgbz.y > 0.f ? gs[6] : 0.f;
            gcol[1] = rgbz.z > 0.f ? gs[7] : 0.f;
            gcol[2] = rgbz.w > 0.f ? gs[8] : 0.f;
            sh_colour_bwd<K>(dxf, dyf, dzf, g.sh, n, i, gcol, gh, 256, gdirf);
            const double gdir[3] = {gdirf[0], gdirf[1], gdirf[2]};
            const double dd = G.dir[0] * gdir[0] + G.dir[1] * gdir[1] + G.dir[2] * gdir[2];
            double gd[3];
            const double idist = 1.0 / G.dist;
            for (int a = 0; a < 3; a++) gd[a] = (gdir[a] - G.dir[a] * dd) * idist;
            for (int a = 0; a < 3; a++) gmu[a] += gd[a];
            // camera centre -R^T t moves by -R^T rho: dL/drho += R dL/d(mu - C)
            for (int a = 0; a < 3; a++) pose[a] += k.R[a][0] * gd[0] + k.R[a][1] * gd[1] + k.R[a][2] * gd[2];
            gop += gs[5];
        }
        if (pose_part) {
            // per-wave partial sums of the pose gradient of this view, component-major
            // [V][6][waves] so that the fixed-order reduction reads them contiguously
            const int64_t wid = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
            const int64_t nw = (int64_t)gridDim.x * 4;
#pragma unroll
            for (int e = 0; e < 6; e++) {
                const float tot = wave_total_f((float)pose[e]);
                if (__lane_id() == e) pose_part[((int64_t)vi * 6 + e) * nw + wid] = (double)tot;
            }
        }
    }
    const bool unfrozen = !seg || (live && seg[i] >= min_seg);
    if (live && row_mask) row_mask[i] = (visible && unfrozen) ? 1 : 0;
    if (!anyvis || !(touched || (FUSED && visible && unfrozen))) return;
    // Sigma = M M^T, M = Rq diag(s): dL/dM = 2 dL/dSigma M
    double qn[4], qnorm, Rq[3][3], sc[3];
    unit_quat(qf, qn, qnorm);
    quat_rot(qn[0], qn[1], qn[2], qn[3], Rq);
    for (int a = 0; a < 3; a++) sc[a] = exp((double)lsf[a]);
    double gRq[3][3];
    float gls[3];
    for (int c = 0; c < 3; c++) {
        double gsc = 0;
        for (int a = 0; a < 3; a++) {
            const double gm = 2.0 * (sym_at(gSig, a, 0) * Rq[0][c] + sym_at(gSig, a, 1) * Rq[1][c] +
                                     sym_at(gSig, a, 2) * Rq[2][c]) * sc[c];
            gsc += gm * Rq[a][c];
            gRq[a][c] = gm * sc[c];
        }
        gls[c] = (float)(gsc * sc[c]);
    }
    // R(q) = (w^2 - |v|^2) I + 2 v v^T + 2 w [v]_x on the unit sphere
    const double w = qn[0], vx = qn[1], vy = qn[2], vz = qn[3];
    const double tr = gRq[0][0] + gRq[1][1] + gRq[2][2];
    const double ax[3] = {gRq[2][1] - gRq[1][2], gRq[0][2] - gRq[2][0], gRq[1][0] - gRq[0][1]};
    const double vv[3] = {vx, vy, vz};
    double gq[4];
    gq[0] = 2.0 * w * tr + 2.0 * (vx * ax[0] + vy * ax[1] + vz * ax[2]);
    for (int a = 0; a < 3; a++) {
        double Gv = 0, GTv = 0;
        for (int b = 0; b < 3; b++) {
            Gv += gRq[a][b] * vv[b];
            GTv += gRq[b][a] * vv[b];
        }
        gq[1 + a] = -2.0 * vv[a] * tr + 2.0 * (Gv + GTv) + 2.0 * w * ax[a];
    }
    const double qd = qn[0] * gq[0] + qn[1] * gq[1] + qn[2] * gq[2] + qn[3] * gq[3];
    float gqf[4];
    for (int a = 0; a < 4; a++) gqf[a] = (float)((gq[a] - qn[a] * qd) / qnorm);
    const float gomf = (float)(gop * o * (1.0 - o));
    if (!FUSED) {
        for (int c = 0; c < 3; c++) out.log_scales[c * n + i] += gls[c];
        for (int a = 0; a < 4; a++) out.quats[a * n + i] += gqf[a];
        for (int a = 0; a < 3; a++) out.means[a * n + i] += (float)gmu[a];
        out.opacity_logits[i] += gomf;
#pragma unroll
        for (int e = 0; e < 3 * K; e++) out.sh[e * n + i] += gh[e * 256];
    } else if (visible && unfrozen) {
        const int step = *adam.step;
        const float bc1 = (float)(1.0 - pow((double)adam.b1, step)), bc2 = (float)(1.0 - pow((double)adam.b2, step));
        float *P0 = const_cast<float *>(g.means), *P1 = const_cast<float *>(g.log_scales);
        float *P2 = const_cast<float *>(g.quats), *P3 = const_cast<float *>(g.opacity_logits);
        float *P4 = const_cast<float *>(g.sh);
        const float b1 = adam.b1, b2 = adam.b2, eps = adam.eps;
        float gg[16], lr[16];
        for (int a = 0; a < 3; a++) gg[a] = (float)gmu[a], lr[a] = adam.lr[0];
        adam_batch<3>(P0, adam.m.means, adam.v.means, i, n, 3, gg, lr, b1, b2, eps, bc1, bc2);
        for (int c = 0; c < 3; c++) gg[c] = gls[c], lr[c] = adam.lr[1];
        adam_batch<3>(P1, adam.m.log_scales, adam.v.log_scales, i, n, 3, gg, lr, b1, b2, eps, bc1, bc2);
        for (int a = 0; a < 4; a++) gg[a] = gqf[a], lr[a] = adam.lr[2];
        adam_batch<4>(P2, adam.m.quats, adam.v.quats, i, n, 4, gg, lr, b1, b2, eps, bc1, bc2);
        gg[0] = gomf, lr[0] = adam.lr[3];
        adam_batch<1>(P3, adam.m.opacity_logits, adam.v.opacity_logits, i, n, 1, gg, lr, b1, b2, eps, bc1, bc2);
        // SH in batches of up to 16 coefficients (rows e = 0..2 are the DC terms)
#pragma unroll
        for (int e0 = 0; e0 < 3 * K; e0 += 16) {
            const int cnt = 3 * K - e0 < 16 ? 3 * K - e0 : 16;
#pragma unroll
            for (int k = 0; k < 16; k++) {
                if (k >= cnt) break;
                gg[k] = gh[(e0 + k) * 256];
                lr[k] = e0 + k < 3 ? adam.lr[4] : adam.lr[5];
            }
            adam_batch<16>(P4, adam.m.sh, adam.v.sh, (int64_t)e0 * n + i, n, cnt, gg, lr, b1, b2, eps, bc1, bc2);
        }
    }
}

// ---- ordered list of the Gaussians visible in at least one view ---------------------------------
__global__ __launch_bounds__(256) void k_vis_any_count(const uint32_t *__restrict__ info, int64_t n, int V,
                                                       uint32_t *__restrict__ bsum) {
    __shared__ uint32_t s_w[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool vis = false;
    if (i < n)
        for (int v = 0; v < V; v++) vis |= info[(int64_t)v * n + i] > 0;
    uint32_t tot;
    block_excl_scan256(vis ? 1u : 0u, s_w, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_vis_any_write(const uint32_t *__restrict__ info, int64_t n, int V,
                                                       const uint32_t *__restrict__ boff, uint32_t *__restrict__ list) {
    __shared__ uint32_t s_w[4];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool vis = false;
    if (i < n)
        for (int v = 0; v < V; v++) vis |= info[(int64_t)v * n + i] > 0;
    const uint32_t pos = boff[blockIdx.x] + block_excl_scan256(vis ? 1u : 0u, s_w, nullptr);
    if (vis) list[pos] = (uint32_t)i;
}

// exclusive scan in place of nb block sums by one 1024-thread block; total -> *total
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t *__restrict__ v, int nb, uint32_t *__restrict__ total) {
    __shared__ uint32_t s_w[16];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        const int idx = base + threadIdx.x;
        const uint32_t x = idx < nb ? v[idx] : 0u;
        const uint32_t inc = wave_incl_scan(x);
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

// dpose[v][e] = sum over waves of the partial sums
// One workgroup of 1024 threads per (view, component): the sum of the per-wave partials of the
// waves that ran (all nw waves, or those covering the first *vcount entries of the visible list).
// Each thread keeps four running sums over the partials w = t, t + 1024, t + 2048, t + 3072 (mod
// 4096) so that four loads are in flight, and the sums meet in a fixed order (pairs, then a wave
// tree, then the 16 waves in order), so this reduction adds no run-dependent rounding of its own.
constexpr int kPoseThreads = 1024;
__global__ __launch_bounds__(kPoseThreads) void k_pose_reduce(const double *__restrict__ part, int64_t nw,
                                                              const uint32_t *__restrict__ vcount,
                                                              double *__restrict__ dpose) {
    __shared__ double s_w[kPoseThreads / 64];
    const int64_t live = vcount ? 4 * ceil_div((int64_t)*vcount, 256) : nw;
    const double *p = part + (int64_t)blockIdx.x * nw;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int64_t w = threadIdx.x;
    for (; w + 3 * kPoseThreads < live; w += 4 * kPoseThreads) {
        a0 += p[w];
        a1 += p[w + kPoseThreads];
        a2 += p[w + 2 * kPoseThreads];
        a3 += p[w + 3 * kPoseThreads];
    }
    if (w < live) a0 += p[w];
    if (w + kPoseThreads < live) a1 += p[w + kPoseThreads];
    if (w + 2 * kPoseThreads < live) a2 += p[w + 2 * kPoseThreads];
    double acc = wave_sum_d((a0 + a1) + (a2 + a3));
    if (__lane_id() == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int k = 0; k < kPoseThreads / 64; k++) t += s_w[k];
        dpose[blockIdx.x] = t;
    }
}

}  // namespace gsr

using namespace gsr;

extern "C" gsr_status gsr_project_launch(const gsr_gaussians *g, const gsr_camera *cams, int V, const gsr_raster *r,
                                         gsr_splat *splats, uint32_t *info, hipStream_t st) {
    const int nb = (int)ceil_div(g->n, 256);
    if (nb == 0) return GSR_OK;
#define GSR_PROJ(D) k_project<D><<<nb, 256, 0, st>>>(*g, cams, V, r->width, r->height, r->tile_w, r->tile_h, splats, info)
    switch (g->sh_degree) {
        case 0: GSR_PROJ(0); break;
        case 1: GSR_PROJ(1); break;
        case 2: GSR_PROJ(2); break;
        default: GSR_PROJ(3); break;
    }
#undef GSR_PROJ
    return last_launch();
}

// Workspace: per-wave pose partials [V][6][waves] (float64), then the per-pair screen-space
// gradients [V*n][10] (float32) summed from the instance records.
static size_t pose_part_bytes(int64_t n, int32_t V) {
    const int64_t nw = 4 * ceil_div(n > 0 ? n : 1, 256);
    return (size_t)((nw * (V > 0 ? V : 1) * 6 * sizeof(double) + 255) & ~(int64_t)255);
}

extern "C" size_t gsr_project_bwd_workspace(int64_t n, int32_t n_views) {
    return pose_part_bytes(n, n_views) +
           (size_t)((n > 0 ? n : 1) * (int64_t)(n_views > 0 ? n_views : 1) * GSR_SPLAT_GRAD_FLOATS * sizeof(float)) + 256;
}

extern "C" gsr_status gsr_pair_grads_launch(const float *, const gsr_emission *, const uint32_t *, int64_t, float *,
                                            bool, hipStream_t);

extern "C" gsr_status gsr_project_bwd_launch(const gsr_gaussians *g, const gsr_camera *cams, int V,
                                             const gsr_raster *r, const gsr_splat *splats, const float *dinst,
                                             const gsr_emission *em, const gsr_param_grads *out,
                                             double *dpose, const uint32_t *tile_info, const int32_t *seg,
                                             int32_t min_seg, uint8_t *row_mask, const gsr_adam_fused *fa,
                                             const uint32_t *vlist, const uint32_t *vcount, void *ws,
                                             hipStream_t st) {
    const int nb = (int)ceil_div(g->n, 256);
    if (nb == 0) {
        if (dpose) {
            // no Gaussians: zero pose gradient
            k_pose_reduce<<<V * 6, kPoseThreads, 0, st>>>(static_cast<double *>(ws), 0, nullptr, dpose);
        }
        return last_launch();
    }
    double *part = dpose ? static_cast<double *>(ws) : nullptr;
    float *dsplat = reinterpret_cast<float *>(static_cast<char *>(ws) + pose_part_bytes(g->n, V));
    gsr_status s = gsr_pair_grads_launch(dinst, em, tile_info, (int64_t)V * g->n, dsplat, false, st);
    if (s != GSR_OK) return s;
    FusedAdam A{};
    gsr_param_grads none{};
    if (fa) {
        A.m = fa->m;
        A.v = fa->v;
        for (int k = 0; k < 6; k++) A.lr[k] = fa->lr[k];
        A.b1 = fa->beta1;
        A.b2 = fa->beta2;
        A.eps = fa->eps;
        A.step = fa->step;
    }
    const gsr_param_grads &O = out ? *out : none;
#define GSR_PB(D, F)                                                                                          \
    k_project_bwd<D, F><<<nb, 256, 0, st>>>(*g, cams, V, r->width, r->height, splats, dsplat, O, part, tile_info, \
                                            seg, min_seg, row_mask, A, vlist, vcount)
#define GSR_PBD(F)                   \
    switch (g->sh_degree) {          \
        case 0: GSR_PB(0, F); break; \
        case 1: GSR_PB(1, F); break; \
        case 2: GSR_PB(2, F); break; \
        default: GSR_PB(3, F); break; \
    }
    if (fa) {
        GSR_PBD(true)
    } else {
        GSR_PBD(false)
    }
#undef GSR_PBD
#undef GSR_PB
    if (dpose) k_pose_reduce<<<V * 6, kPoseThreads, 0, st>>>(part, 4 * (int64_t)nb, vlist ? vcount : nullptr, dpose);
    return last_launch();
}

extern "C" size_t gsr_visible_list_ws_bytes(int64_t n) { return (size_t)(ceil_div(n > 0 ? n : 1, 256) * 4 + 256); }

extern "C" gsr_status gsr_visible_list_launch(const uint32_t *info, int64_t n, int V, uint32_t *list, uint32_t *count,
                                              void *ws, hipStream_t st) {
    const int nb = (int)ceil_div(n > 0 ? n : 1, 256);
    uint32_t *bsum = static_cast<uint32_t *>(ws);
    k_vis_any_count<<<nb, 256, 0, st>>>(info, n, V, bsum);
    k_scan_blocks<<<1, 1024, 0, st>>>(bsum, nb, count);
    k_vis_any_write<<<nb, 256, 0, st>>>(info, n, V, bsum, list);
    return last_launch();
}

// ---- visible list without a workspace argument -------------------------------------------------
// The block counts of gsr_visible_list live in a file-scope device array instead of a caller's
// workspace.  Every GPU the library runs on holds its own copy until the process ends; its address
// on each device is looked up once (hipGetSymbolAddress with that device current) and kept, and
// only that address is ever handed to kernels.  Each of the first ceil(n / 256) words is written
// by k_vis_any_count before k_scan_blocks reads it, so nothing has to be cleared between calls.
namespace {
constexpr int64_t kNoAllocMaxN = int64_t(1) << 24;  // 16,777,216 Gaussians
constexpr size_t kNoAllocWords = (size_t)(kNoAllocMaxN / 256) + 64;
static_assert(kNoAllocWords * 4 >= (size_t)((kNoAllocMaxN / 256) * 4 + 256), "scratch covers the block counts");
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint32_t scratch[kNoAllocWords];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's copy of the scratch array (nullptr on a HIP error).
void *scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int64_t gsr_visible_list_noalloc_max(void) { return kNoAllocMaxN; }

extern "C" gsr_status gsr_visible_list_noalloc(const uint32_t *tile_info, int64_t n, int32_t n_views, uint32_t *list,
                                               uint32_t *count, gsr_stream stream) {
    if (n < 0 || n_views < 1 || !count || (n > 0 && (!tile_info || !list))) return GSR_E_INVALID;
    if (n > kNoAllocMaxN) return GSR_E_CAPACITY;
    void *ws = scratch_on_current_device();
    if (!ws) return GSR_E_HIP;
    return gsr_visible_list_launch(tile_info, n, n_views, list, count, ws, static_cast<hipStream_t>(stream));
}
