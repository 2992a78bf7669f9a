// EWA projection of 3-D Gaussians into pinhole views, and its exact backward with the camera-pose
// gradient.  One thread per Gaussian walks every view, so the per-Gaussian parameters (up to 236
// bytes at SH degree 3) are read from HBM once per step instead of once per view, and the
// parameter gradients are accumulated over views in registers (no atomics, no re-reads).
// The arithmetic is double precision: the stage is bound by HBM traffic, and FP64 keeps the
// screen-space results within a rounding of the exact values of the float32 inputs.
#include "gsr_internal.h"

namespace gsr {

// Real spherical harmonics without Condon-Shortley phase, orthonormal, (l, m=-l..l) order, as
// polynomials of the unit direction (x, y, z); dY gets the polynomial gradient.
template <int DEG, bool GRAD>
__device__ __forceinline__ void sh_basis(double x, double y, double z, double *Y, double (*dY)[3]) {
    Y[0] = 0.28209479177387814;
    if (GRAD) { dY[0][0] = dY[0][1] = dY[0][2] = 0.0; }
    if (DEG >= 1) {
        const double a = 0.4886025119029199;
        Y[1] = a * y; Y[2] = a * z; Y[3] = a * x;
        if (GRAD) {
            dY[1][0] = 0; dY[1][1] = a; dY[1][2] = 0;
            dY[2][0] = 0; dY[2][1] = 0; dY[2][2] = a;
            dY[3][0] = a; dY[3][1] = 0; dY[3][2] = 0;
        }
    }
    if (DEG >= 2) {
        const double b = 1.0925484305920792, c = 0.31539156525252005, d = 0.5462742152960396;
        Y[4] = b * x * y; Y[5] = b * y * z; Y[6] = c * (3.0 * z * z - 1.0); Y[7] = b * x * z;
        Y[8] = d * (x * x - y * y);
        if (GRAD) {
            dY[4][0] = b * y; dY[4][1] = b * x; dY[4][2] = 0;
            dY[5][0] = 0; dY[5][1] = b * z; dY[5][2] = b * y;
            dY[6][0] = 0; dY[6][1] = 0; dY[6][2] = 6.0 * c * z;
            dY[7][0] = b * z; dY[7][1] = 0; dY[7][2] = b * x;
            dY[8][0] = 2.0 * d * x; dY[8][1] = -2.0 * d * y; dY[8][2] = 0;
        }
    }
    if (DEG >= 3) {
        const double e = 0.5900435899266435, f = 2.890611442640554, g = 0.4570457994644658;
        const double h = 0.3731763325901154, k = 1.445305721320277;
        const double x2 = x * x, y2 = y * y, z2 = z * z;
        Y[9] = e * y * (3.0 * x2 - y2);
        Y[10] = f * x * y * z;
        Y[11] = g * y * (5.0 * z2 - 1.0);
        Y[12] = h * z * (5.0 * z2 - 3.0);
        Y[13] = g * x * (5.0 * z2 - 1.0);
        Y[14] = k * z * (x2 - y2);
        Y[15] = e * x * (x2 - 3.0 * y2);
        if (GRAD) {
            dY[9][0] = 6.0 * e * x * y; dY[9][1] = 3.0 * e * (x2 - y2); dY[9][2] = 0;
            dY[10][0] = f * y * z; dY[10][1] = f * x * z; dY[10][2] = f * x * y;
            dY[11][0] = 0; dY[11][1] = g * (5.0 * z2 - 1.0); dY[11][2] = 10.0 * g * y * z;
            dY[12][0] = 0; dY[12][1] = 0; dY[12][2] = h * (15.0 * z2 - 3.0);
            dY[13][0] = g * (5.0 * z2 - 1.0); dY[13][1] = 0; dY[13][2] = 10.0 * g * x * z;
            dY[14][0] = 2.0 * k * x * z; dY[14][1] = -2.0 * k * y * z; dY[14][2] = k * (x2 - y2);
            dY[15][0] = 3.0 * e * (x2 - y2); dY[15][1] = -6.0 * e * x * y; dY[15][2] = 0;
        }
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

// Everything the forward and backward share for one (view, Gaussian).
struct ViewGeom {
    double p[3];        // camera-frame mean
    double Sc[3][3];    // camera-frame covariance
    double j00, j02, j11, j12, tx, ty;
    bool clx, cly;
    double a, b, c;     // Sigma' = [[a, b], [b, c]]
    double det;
    double u, v;
    double dir[3], dist;
};

__device__ __forceinline__ bool view_geom(const double mu[3], const double Sig[3][3], const Cam &k, int W, int H,
                                          ViewGeom &G) {
    for (int a = 0; a < 3; a++) G.p[a] = k.R[a][0] * mu[0] + k.R[a][1] * mu[1] + k.R[a][2] * mu[2] + k.t[a];
    const double z = G.p[2];
    if (!(z > k.znear)) return false;
    double RS[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) RS[a][b] = k.R[a][0] * Sig[0][b] + k.R[a][1] * Sig[1][b] + k.R[a][2] * Sig[2][b];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) G.Sc[a][b] = RS[a][0] * k.R[b][0] + RS[a][1] * k.R[b][1] + RS[a][2] * k.R[b][2];
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
    const double r0[3] = {G.j00 * G.Sc[0][0] + G.j02 * G.Sc[2][0], G.j00 * G.Sc[0][1] + G.j02 * G.Sc[2][1],
                          G.j00 * G.Sc[0][2] + G.j02 * G.Sc[2][2]};
    const double r1[3] = {G.j11 * G.Sc[1][0] + G.j12 * G.Sc[2][0], G.j11 * G.Sc[1][1] + G.j12 * G.Sc[2][1],
                          G.j11 * G.Sc[1][2] + G.j12 * G.Sc[2][2]};
    G.a = r0[0] * G.j00 + r0[2] * G.j02 + GSR_LOWPASS;
    G.b = r0[1] * G.j11 + r0[2] * G.j12;
    G.c = r1[1] * G.j11 + r1[2] * G.j12 + GSR_LOWPASS;
    G.det = G.a * G.c - G.b * G.b;
    G.u = k.fx * G.p[0] * iz + k.cx;
    G.v = k.fy * G.p[1] * iz + k.cy;
    double d[3] = {mu[0] - k.C[0], mu[1] - k.C[1], mu[2] - k.C[2]};
    G.dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int a = 0; a < 3; a++) G.dir[a] = d[a] / G.dist;
    return true;
}

__device__ __forceinline__ void gaussian_cov(const gsr_gaussians &g, int64_t i, double mu[3], double Rq[3][3],
                                             double s[3], double qn[4], double &qnorm, double Sig[3][3]) {
    const int64_t n = g.n;
    for (int a = 0; a < 3; a++) mu[a] = g.means[a * n + i];
    double q[4];
    for (int a = 0; a < 4; a++) q[a] = g.quats[a * n + i];
    qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int a = 0; a < 4; a++) qn[a] = q[a] / qnorm;
    quat_rot(qn[0], qn[1], qn[2], qn[3], Rq);
    for (int a = 0; a < 3; a++) s[a] = exp((double)g.log_scales[a * n + i]);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b <= a; b++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += Rq[a][k] * Rq[b][k] * s[k] * s[k];
            Sig[a][b] = Sig[b][a] = acc;
        }
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
    double mu[3], Rq[3][3], s[3], qn[4], qnorm, Sig[3][3];
    gaussian_cov(g, i, mu, Rq, s, qn, qnorm, Sig);
    const double o = 1.0 / (1.0 + exp(-(double)g.opacity_logits[i]));
    float h[3 * K];
#pragma unroll
    for (int e = 0; e < 3 * K; e++) h[e] = g.sh[e * n + i];
    for (int vi = 0; vi < V; vi++) {
        Cam k;
        load_cam(cams[vi], k);
        const int64_t gid = vi * n + i;
        ViewGeom G;
        uint32_t ntiles = 0, zbits = 0, r0 = 0, r1 = 0;
        double4 rec0 = make_double4(0, 0, 0, 0);
        float4 rec1 = make_float4(0, 0, 0, 0), rec2 = make_float4(0, 0, 0, 0);
        if (view_geom(mu, Sig, k, W, H, G) && 255.0 * o >= 1.0) {
            // colour in the viewing direction
            double Y[K];
            sh_basis<DEG, false>(G.dir[0], G.dir[1], G.dir[2], Y, nullptr);
            float col[3];
            for (int ch = 0; ch < 3; ch++) {
                double acc = 0.5;
#pragma unroll
                for (int kk = 0; kk < K; kk++) acc += Y[kk] * (double)h[3 * kk + ch];
                col[ch] = (float)(acc > 0.0 ? acc : 0.0);
            }
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
                // Cholesky factor of kappa Q, Q = [[c, -b], [-b, a]] / det:
                // l11 = sqrt(kappa c / det), l21 = -kappa b / (det l11), l22 = sqrt(kappa / c)
                const double qa = GSR_KAPPA * G.c / G.det, qb = -GSR_KAPPA * G.b / G.det;
                const double l11 = sqrt(qa);
                rec0 = make_double4(G.u, G.v, 0, 0);
                rec1 = make_float4((float)l11, (float)(qb / l11), (float)sqrt(GSR_KAPPA / G.c), (float)o);
                rec2 = make_float4(zf, col[0], col[1], col[2]);
            }
        }
        // only visible pairs are ever read back: skip the record writes of the others
        info[gid] = ntiles;
        if (ntiles) {
            double2 *dst = reinterpret_cast<double2 *>(splats + gid);
            dst[0] = make_double2(rec0.x, rec0.y);
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
__device__ __forceinline__ void block_sum6_d(double v[6], double *s_red /*[4][6]*/, double *out) {
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 6; e++) {
        double r = wave_sum_d(v[e]);
        if (__lane_id() == 0) s_red[w * 6 + e] = r;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double acc = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); k++) acc += s_red[k * 6 + threadIdx.x];
        out[threadIdx.x] = acc;
    }
    __syncthreads();
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd(gsr_gaussians g, const gsr_camera *__restrict__ cams, int V,
                                                     int W, int H, float *__restrict__ dsplat,
                                                     gsr_param_grads out, double *__restrict__ pose_part,
                                                     const uint32_t *__restrict__ tile_info,
                                                     const int32_t *__restrict__ seg, int32_t min_seg,
                                                     uint8_t *__restrict__ row_mask) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    __shared__ double s_red[4 * 6];
    const int64_t n = g.n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;
    double mu[3] = {0, 0, 0}, Rq[3][3], s[3] = {1, 1, 1}, qn[4] = {1, 0, 0, 0}, qnorm = 1, Sig[3][3];
    double o = 0;
    float h[3 * K];
    if (live) {
        gaussian_cov(g, i, mu, Rq, s, qn, qnorm, Sig);
        o = 1.0 / (1.0 + exp(-(double)g.opacity_logits[i]));
#pragma unroll
        for (int e = 0; e < 3 * K; e++) h[e] = g.sh[e * n + i];
    }
    double gSig[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double gmu[3] = {0, 0, 0}, gop = 0;
    float gh[3 * K];
#pragma unroll
    for (int e = 0; e < 3 * K; e++) gh[e] = 0.f;
    bool touched = false, visible = false;

    for (int vi = 0; vi < V; vi++) {
        double pose[6] = {0, 0, 0, 0, 0, 0};
        float gs[10];
        bool any = false;
        if (live) {
            // with tile_info, only the pairs that were rendered can hold gradients: read those and
            // reset them, leaving dsplat zeroed for the next backward without a separate fill
            const bool vis = tile_info ? tile_info[(int64_t)vi * n + i] > 0 : true;
            visible |= vis;
            if (vis) {
                float *src = dsplat + ((int64_t)vi * n + i) * GSR_SPLAT_GRAD_FLOATS;
                float2 *s2 = reinterpret_cast<float2 *>(src);
#pragma unroll
                for (int e = 0; e < 5; e++) {
                    const float2 q = s2[e];
                    gs[2 * e] = q.x;
                    gs[2 * e + 1] = q.y;
                }
#pragma unroll
                for (int e = 0; e < 10; e++) any |= gs[e] != 0.f;
                if (tile_info && any) {
#pragma unroll
                    for (int e = 0; e < 5; e++) s2[e] = make_float2(0.f, 0.f);
                }
            }
        }
        Cam k;
        load_cam(cams[vi], k);
        ViewGeom G;
        if (any && view_geom(mu, Sig, k, W, H, G)) {
            touched = true;
            const double x = G.p[0], y = G.p[1], z = G.p[2], iz = 1.0 / z;
            // conic Q = [[c, -b], [-b, a]] / det
            const double Qa = G.c / G.det, Qb = -G.b / G.det, Qc = G.a / G.det;
            // dL/dSigma' = -Q dL/dQ Q with the symmetric dL/dQ = [[ga, gb/2], [gb/2, gc]]
            const double ga = gs[2], gb = 0.5 * gs[3], gc = gs[4];
            const double m00 = Qa * ga + Qb * gb, m01 = Qa * gb + Qb * gc;
            const double m10 = Qb * ga + Qc * gb, m11 = Qb * gb + Qc * gc;
            const double S00 = -(m00 * Qa + m01 * Qb), S01 = -(m00 * Qb + m01 * Qc);
            const double S11 = -(m10 * Qb + m11 * Qc);
            // J rows: J0 = (j00, 0, j02), J1 = (0, j11, j12)
            const double J0[3] = {G.j00, 0.0, G.j02}, J1[3] = {0.0, G.j11, G.j12};
            // dL/dSc = J^T dL/dSigma' J
            double gSc[3][3];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    gSc[a][b] = J0[a] * (S00 * J0[b] + S01 * J1[b]) + J1[a] * (S01 * J0[b] + S11 * J1[b]);
            // dL/dJ = 2 dL/dSigma' J Sc (rows 0 and 1)
            double JS0[3], JS1[3];
            for (int b = 0; b < 3; b++) {
                JS0[b] = J0[0] * G.Sc[0][b] + J0[2] * G.Sc[2][b];
                JS1[b] = J1[1] * G.Sc[1][b] + J1[2] * G.Sc[2][b];
            }
            const double gJ00 = 2.0 * (S00 * JS0[0] + S01 * JS1[0]);
            const double gJ02 = 2.0 * (S00 * JS0[2] + S01 * JS1[2]);
            const double gJ11 = 2.0 * (S01 * JS0[1] + S11 * JS1[1]);
            const double gJ12 = 2.0 * (S01 * JS0[2] + S11 * JS1[2]);
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
            double T1[3][3];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    T1[a][b] = k.R[0][a] * gSc[0][b] + k.R[1][a] * gSc[1][b] + k.R[2][a] * gSc[2][b];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    gSig[a][b] += T1[a][0] * k.R[0][b] + T1[a][1] * k.R[1][b] + T1[a][2] * k.R[2][b];
            // pose, rotation part through Sc: <dL/dSc, [e]x Sc - Sc [e]x> = 2 tr([e]x Sc dL/dSc)
            double A[3][3];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    A[a][b] = G.Sc[a][0] * gSc[0][b] + G.Sc[a][1] * gSc[1][b] + G.Sc[a][2] * gSc[2][b];
            pose[3] += 2.0 * (A[1][2] - A[2][1]);
            pose[4] += 2.0 * (A[2][0] - A[0][2]);
            pose[5] += 2.0 * (A[0][1] - A[1][0]);
            // p = R mu + t
            for (int a = 0; a < 3; a++) gmu[a] += k.R[0][a] * gp[0] + k.R[1][a] * gp[1] + k.R[2][a] * gp[2];
            for (int a = 0; a < 3; a++) pose[a] += gp[a];
            pose[3] += y * gp[2] - z * gp[1];
            pose[4] += z * gp[0] - x * gp[2];
            pose[5] += x * gp[1] - y * gp[0];
            // colour: clamp at zero, SH coefficients, viewing direction
            double Y[K], dY[K][3];
            sh_basis<DEG, true>(G.dir[0], G.dir[1], G.dir[2], Y, dY);
            double gdir[3] = {0, 0, 0};
            for (int ch = 0; ch < 3; ch++) {
                double pre = 0.5;
#pragma unroll
                for (int kk = 0; kk < K; kk++) pre += Y[kk] * (double)h[3 * kk + ch];
                if (!(pre > 0.0)) continue;
                const double gcol = gs[6 + ch];
#pragma unroll
                for (int kk = 0; kk < K; kk++) {
                    gh[3 * kk + ch] += (float)(gcol * Y[kk]);
                    for (int a = 0; a < 3; a++) gdir[a] += gcol * h[3 * kk + ch] * dY[kk][a];
                }
            }
            const double dd = G.dir[0] * gdir[0] + G.dir[1] * gdir[1] + G.dir[2] * gdir[2];
            double gd[3];
            for (int a = 0; a < 3; a++) gd[a] = (gdir[a] - G.dir[a] * dd) / G.dist;
            for (int a = 0; a < 3; a++) gmu[a] += gd[a];
            // camera centre -R^T t moves by -R^T rho: dL/drho += R dL/d(mu - C)
            for (int a = 0; a < 3; a++) pose[a] += k.R[a][0] * gd[0] + k.R[a][1] * gd[1] + k.R[a][2] * gd[2];
            gop += gs[5];
        }
        if (pose_part) {
            // deterministic per-block partial sums of the pose gradient of this view
            block_sum6_d(pose, s_red, pose_part + ((int64_t)blockIdx.x * V + vi) * 6);
        }
    }
    if (live && row_mask) row_mask[i] = (visible && (!seg || seg[i] >= min_seg)) ? 1 : 0;
    if (!live || !touched) return;
    // Sigma = M M^T, M = Rq diag(s): dL/dM = 2 dL/dSigma M
    double gRq[3][3];
    for (int c = 0; c < 3; c++) {
        double gsc = 0;
        for (int a = 0; a < 3; a++) {
            const double gm = 2.0 * (gSig[a][0] * Rq[0][c] + gSig[a][1] * Rq[1][c] + gSig[a][2] * Rq[2][c]) * s[c];
            gsc += gm * Rq[a][c];
            gRq[a][c] = gm * s[c];
        }
        out.log_scales[c * n + i] += (float)(gsc * s[c]);
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
    for (int a = 0; a < 4; a++) out.quats[a * n + i] += (float)((gq[a] - qn[a] * qd) / qnorm);
    for (int a = 0; a < 3; a++) out.means[a * n + i] += (float)gmu[a];
    out.opacity_logits[i] += (float)(gop * o * (1.0 - o));
#pragma unroll
    for (int e = 0; e < 3 * K; e++) out.sh[e * n + i] += gh[e];
}

// dpose[v][e] = sum over blocks of the partial sums (fixed order: deterministic)
__global__ void k_pose_reduce(const double *__restrict__ part, int nblocks, int V, double *__restrict__ dpose) {
    const int v = blockIdx.x;
    const int e = threadIdx.x >> 6;  // 6 waves, one per component
    if (e >= 6) return;
    double acc = 0;
    for (int b = __lane_id(); b < nblocks; b += 64) acc += part[((int64_t)b * V + v) * 6 + e];
    acc = wave_sum_d(acc);
    if (__lane_id() == 0) dpose[v * 6 + e] = acc;
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

extern "C" size_t gsr_project_bwd_workspace(int64_t n, int32_t n_views) {
    const int64_t nb = ceil_div(n > 0 ? n : 1, 256);
    return (size_t)(nb * (n_views > 0 ? n_views : 1) * 6 * sizeof(double) + 256);
}

extern "C" gsr_status gsr_project_bwd_launch(const gsr_gaussians *g, const gsr_camera *cams, int V,
                                             const gsr_raster *r, float *dsplat, const gsr_param_grads *out,
                                             double *dpose, const uint32_t *tile_info, const int32_t *seg,
                                             int32_t min_seg, uint8_t *row_mask, void *ws, hipStream_t st) {
    const int nb = (int)ceil_div(g->n, 256);
    if (nb == 0) {
        if (dpose) {
            // no Gaussians: zero pose gradient
            k_pose_reduce<<<V, 384, 0, st>>>(static_cast<double *>(ws), 0, V, dpose);
        }
        return last_launch();
    }
    double *part = dpose ? static_cast<double *>(ws) : nullptr;
#define GSR_PB(D)                                                                                          \
    k_project_bwd<D><<<nb, 256, 0, st>>>(*g, cams, V, r->width, r->height, dsplat, *out, part, tile_info, seg, \
                                         min_seg, row_mask)
    switch (g->sh_degree) {
        case 0: GSR_PB(0); break;
        case 1: GSR_PB(1); break;
        case 2: GSR_PB(2); break;
        default: GSR_PB(3); break;
    }
#undef GSR_PB
    if (dpose) k_pose_reduce<<<V, 384, 0, st>>>(part, nb, V, dpose);
    return last_launch();
}
