// Gaussian-based loop registration (Sec. III-D, Eq. 13-16).
//
// Prepare: the source set (the loopframe's segment) and the target set of Eq. 13 (Gaussians that
// some query keyframe sees inside its image with its centre within d_max) are flagged per row and
// compacted in row order; every listed Gaussian gets its planar regularised covariance (eigenvalues
// replaced by 1, 1, 1e-3, the small one on the smallest-scale axis: I - 0.999 a a^T); the target
// means go into a hashed cell grid of edge slightly above d_corr.
//
// Iterate (Gauss-Newton, all on the device): one lane per source Gaussian moves its mean by the
// current pose, finds the nearest target mean within d_corr among the 27 neighbouring cells,
// forms r = mu_n - q, C = S_n + R S_m R^T, W = C^-1 and J = [-I, [q]x], and accumulates
// J^T W J, J^T W r, r^T W r and |r|^2 in float64; blocks write partials, one block adds them in a
// fixed order, solves the 6x6 system by Cholesky and applies the left update
// (R, t) <- (Exp(phi) R, Exp(phi) t + rho).  Converged or failed iterations turn the remaining
// launches into no-ops, so a fixed number of iterations can be queued without host round trips.
//
// The geometric decisions (frustum test, distances, nearest neighbour) use float64 operations
// rounded one by one in a stated order, so another implementation can reproduce them exactly.
#include "grid.h"

extern "C" gsr_status gsr_scan_launch(const uint32_t *, int64_t, uint32_t *, uint32_t *, void *, hipStream_t);
extern "C" size_t gsr_scan_ws_bytes(int64_t);
extern "C" size_t gsr_sort_pairs_ws_bytes(int64_t);
extern "C" gsr_status gsr_fill_u32_launch(void *, uint32_t, int64_t, hipStream_t);

namespace gsr {

constexpr int kGicpAcc = 30;  // H (21, upper triangle row-major), g (6), cost, |r|^2, count
enum { kStCost = 27, kStSq = 28, kStCount = 29, kStXi = 30, kStConv = 36, kStIters = 37, kStFailed = 38 };
constexpr double kRegSmall = 1e-3;
constexpr double kEpsRho = 2.5e-3, kEpsPhi = 2.5e-4;

__device__ __forceinline__ double dmadd3(double a0, double b0, double a1, double b1, double a2, double b2) {
    // ((a0 b0 + a1 b1) + a2 b2), each operation rounded
    return __dadd_rn(__dadd_rn(__dmul_rn(a0, b0), __dmul_rn(a1, b1)), __dmul_rn(a2, b2));
}

__global__ void k_gicp_flags(const float *__restrict__ means, const int32_t *__restrict__ seg, int64_t n,
                             int32_t src_segment, const gsr_camera *__restrict__ cams, int n_cams, double dd_max,
                             uint32_t *__restrict__ f_src, uint32_t *__restrict__ f_tgt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool src = seg[i] == src_segment;
    bool tgt = false;
    const double mx = means[i], my = means[n + i], mz = means[2 * n + i];
    for (int k = 0; k < n_cams && !src && !tgt; k++) {
        const gsr_camera &c = cams[k];
        double R[9], t[3];
        for (int e = 0; e < 9; e++) R[e] = c.R[e];
        for (int e = 0; e < 3; e++) t[e] = c.t[e];
        const double x = __dadd_rn(dmadd3(R[0], mx, R[1], my, R[2], mz), t[0]);
        const double y = __dadd_rn(dmadd3(R[3], mx, R[4], my, R[5], mz), t[1]);
        const double z = __dadd_rn(dmadd3(R[6], mx, R[7], my, R[8], mz), t[2]);
        if (!(z > (double)c.z_near)) continue;
        const double u = __dadd_rn(__dmul_rn((double)c.fx, __ddiv_rn(x, z)), (double)c.cx);
        const double v = __dadd_rn(__dmul_rn((double)c.fy, __ddiv_rn(y, z)), (double)c.cy);
        if (!(u >= 0.0 && u < (double)c.width && v >= 0.0 && v < (double)c.height)) continue;
        // centre -R^T t
        const double cx = -dmadd3(R[0], t[0], R[3], t[1], R[6], t[2]);
        const double cy = -dmadd3(R[1], t[0], R[4], t[1], R[7], t[2]);
        const double cz = -dmadd3(R[2], t[0], R[5], t[1], R[8], t[2]);
        tgt = sqdist_rn(mx, my, mz, cx, cy, cz) < dd_max;
    }
    f_src[i] = src ? 1u : 0u;
    f_tgt[i] = tgt ? 1u : 0u;
}

__global__ void k_gicp_compact(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ off, int64_t n,
                               uint32_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) out[off[i]] = (uint32_t)i;
}

// cov [6][cap] (xx, xy, xz, yy, yz, zz) of the listed Gaussians
__global__ void k_gicp_cov(const uint32_t *__restrict__ list, const uint32_t *__restrict__ count, int64_t cap,
                           const float *__restrict__ quats, const float *__restrict__ log_scales, int64_t n,
                           double *__restrict__ cov) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (int64_t)*count || j >= cap) return;
    const int64_t i = list[j];
    double w = quats[i], x = quats[n + i], y = quats[2 * n + i], z = quats[3 * n + i];
    const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= inv, x *= inv, y *= inv, z *= inv;
    const float s0 = log_scales[i], s1 = log_scales[n + i], s2 = log_scales[2 * n + i];
    const int a = (s1 < s0 && s1 <= s2) ? 1 : ((s2 < s0 && s2 < s1) ? 2 : 0);  // first smallest
    double ax, ay, az;  // column a of the rotation
    if (a == 0) ax = 1 - 2 * (y * y + z * z), ay = 2 * (x * y + w * z), az = 2 * (x * z - w * y);
    else if (a == 1) ax = 2 * (x * y - w * z), ay = 1 - 2 * (x * x + z * z), az = 2 * (y * z + w * x);
    else ax = 2 * (x * z + w * y), ay = 2 * (y * z - w * x), az = 1 - 2 * (x * x + y * y);
    const double k = 1.0 - kRegSmall;
    cov[j] = 1.0 - k * ax * ax;
    cov[cap + j] = -k * ax * ay;
    cov[2 * cap + j] = -k * ax * az;
    cov[3 * cap + j] = 1.0 - k * ay * ay;
    cov[4 * cap + j] = -k * ay * az;
    cov[5 * cap + j] = 1.0 - k * az * az;
}

// Target means in grid order (x, y, z as float, list position as bits), so that a probe scans a
// cell's candidates contiguously instead of gathering them through two index arrays.
__global__ void k_gicp_grid_points(const float *__restrict__ means, int64_t n, const uint32_t *__restrict__ tgt_list,
                                   const uint32_t *__restrict__ counts, const uint32_t *__restrict__ val,
                                   float4 *__restrict__ gp) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)counts[1]) return;
    const uint32_t p = val[e];
    const int64_t i = tgt_list[p];
    gp[e] = make_float4(means[i], means[n + i], means[2 * n + i], __uint_as_float(p));
}

__device__ __forceinline__ int tri(int i, int j) { return i * 6 - i * (i - 1) / 2 + (j - i); }  // i <= j

__device__ __forceinline__ bool gicp_stopped(const double *stats) {
    return stats[kStConv] != 0.0 || stats[kStFailed] != 0.0;
}

// One linearisation: per-block partial sums of (H, g, cost, |r|^2, count).
__global__ __launch_bounds__(256) void k_gicp_linearise(
    const float *__restrict__ means, int64_t n, const uint32_t *__restrict__ src_list,
    const uint32_t *__restrict__ tgt_list, const uint32_t *__restrict__ counts, const double *__restrict__ src_cov,
    const double *__restrict__ tgt_cov, int64_t cap, const uint32_t *__restrict__ key, const uint32_t *__restrict__ val,
    const uint32_t *__restrict__ bucket, const float4 *__restrict__ gp, double inv_cell, double dd_corr,
    const double *__restrict__ pose, const double *__restrict__ stats, double *__restrict__ partial,
    int32_t *__restrict__ corr) {
    __shared__ double s_acc[4][kGicpAcc];
    if (gicp_stopped(stats)) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n_src = counts[0];
    const uint32_t n_tgt = counts[1];
    double acc[kGicpAcc];
#pragma unroll
    for (int e = 0; e < kGicpAcc; e++) acc[e] = 0.0;
    if (j < n_src) {
        double R[9], t[3];
        for (int e = 0; e < 9; e++) R[e] = pose[e];
        for (int e = 0; e < 3; e++) t[e] = pose[9 + e];
        const int64_t i = src_list[j];
        const double mx = means[i], my = means[n + i], mz = means[2 * n + i];
        const double q[3] = {__dadd_rn(dmadd3(R[0], mx, R[1], my, R[2], mz), t[0]),
                             __dadd_rn(dmadd3(R[3], mx, R[4], my, R[5], mz), t[1]),
                             __dadd_rn(dmadd3(R[6], mx, R[7], my, R[8], mz), t[2])};
        const int64_t cx = cell_of(q[0], inv_cell), cy = cell_of(q[1], inv_cell), cz = cell_of(q[2], inv_cell);
        double best = dd_corr;
        uint32_t bi = 0xFFFFFFFFu;
        for (int d = 0; d < 27; d++) {
            const uint32_t h = cell_hash(cx + d % 3 - 1, cy + (d / 3) % 3 - 1, cz + d / 9 - 1);
            for (uint32_t e = grid_lower_bound(key, bucket, h); e < n_tgt && key[e] == h; e++) {
                const float4 c = gp[e];
                const uint32_t p = __float_as_uint(c.w);
                const double d2 = sqdist_rn(c.x, c.y, c.z, q[0], q[1], q[2]);
                if (d2 < best || (d2 == best && p < bi && bi != 0xFFFFFFFFu)) {
                    best = d2;
                    bi = p;
                }
            }
        }
        if (corr) corr[j] = bi == 0xFFFFFFFFu ? -1 : (int32_t)bi;
        if (bi != 0xFFFFFFFFu) {
            const int64_t it = tgt_list[bi];
            const double r[3] = {means[it] - q[0], means[n + it] - q[1], means[2 * n + it] - q[2]};
            // C = S_n + R S_m R^T
            const double Sm[9] = {src_cov[j], src_cov[cap + j], src_cov[2 * cap + j],
                                  src_cov[cap + j], src_cov[3 * cap + j], src_cov[4 * cap + j],
                                  src_cov[2 * cap + j], src_cov[4 * cap + j], src_cov[5 * cap + j]};
            double RS[9], C[9];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    RS[3 * a + b] = R[3 * a] * Sm[b] + R[3 * a + 1] * Sm[3 + b] + R[3 * a + 2] * Sm[6 + b];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    C[3 * a + b] = RS[3 * a] * R[3 * b] + RS[3 * a + 1] * R[3 * b + 1] + RS[3 * a + 2] * R[3 * b + 2];
            const int64_t pb = bi;
            C[0] += tgt_cov[pb], C[1] += tgt_cov[cap + pb], C[2] += tgt_cov[2 * cap + pb];
            C[3] += tgt_cov[cap + pb], C[4] += tgt_cov[3 * cap + pb], C[5] += tgt_cov[4 * cap + pb];
            C[6] += tgt_cov[2 * cap + pb], C[7] += tgt_cov[4 * cap + pb], C[8] += tgt_cov[5 * cap + pb];
            // W = C^-1 (adjugate over determinant)
            double W[9];
            W[0] = C[4] * C[8] - C[5] * C[7];
            W[1] = C[2] * C[7] - C[1] * C[8];
            W[2] = C[1] * C[5] - C[2] * C[4];
            W[3] = C[5] * C[6] - C[3] * C[8];
            W[4] = C[0] * C[8] - C[2] * C[6];
            W[5] = C[2] * C[3] - C[0] * C[5];
            W[6] = C[3] * C[7] - C[4] * C[6];
            W[7] = C[1] * C[6] - C[0] * C[7];
            W[8] = C[0] * C[4] - C[1] * C[3];
            const double id = 1.0 / (C[0] * W[0] + C[1] * W[3] + C[2] * W[6]);
            for (int e = 0; e < 9; e++) W[e] *= id;
            // J = [-I, [q]x]: column c of J
            double J[3][6];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) J[a][b] = a == b ? -1.0 : 0.0;
            J[0][3] = 0.0, J[0][4] = -q[2], J[0][5] = q[1];
            J[1][3] = q[2], J[1][4] = 0.0, J[1][5] = -q[0];
            J[2][3] = -q[1], J[2][4] = q[0], J[2][5] = 0.0;
            double WJ[3][6], Wr[3];
            for (int a = 0; a < 3; a++) {
                for (int c = 0; c < 6; c++) WJ[a][c] = W[3 * a] * J[0][c] + W[3 * a + 1] * J[1][c] + W[3 * a + 2] * J[2][c];
                Wr[a] = W[3 * a] * r[0] + W[3 * a + 1] * r[1] + W[3 * a + 2] * r[2];
            }
            for (int a = 0; a < 6; a++) {
                for (int b = a; b < 6; b++) acc[tri(a, b)] = J[0][a] * WJ[0][b] + J[1][a] * WJ[1][b] + J[2][a] * WJ[2][b];
                acc[21 + a] = J[0][a] * Wr[0] + J[1][a] * Wr[1] + J[2][a] * Wr[2];
            }
            acc[kStCost] = r[0] * Wr[0] + r[1] * Wr[1] + r[2] * Wr[2];
            acc[kStSq] = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            acc[kStCount] = 1.0;
        }
    }
#pragma unroll
    for (int e = 0; e < kGicpAcc; e++) acc[e] = wave_sum_d(acc[e]);
    if (lane_id() == 0)
        for (int e = 0; e < kGicpAcc; e++) s_acc[threadIdx.x >> 6][e] = acc[e];
    __syncthreads();
    if (threadIdx.x < kGicpAcc) {
        const int e = threadIdx.x;
        partial[(int64_t)blockIdx.x * kGicpAcc + e] = (s_acc[0][e] + s_acc[1][e]) + (s_acc[2][e] + s_acc[3][e]);
    }
}

__device__ void so3_exp(const double phi[3], double E[9]) {
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = sqrt(th2);
    const double K[9] = {0.0, -phi[2], phi[1], phi[2], 0.0, -phi[0], -phi[1], phi[0], 0.0};
    double a = 1.0, b = 0.0;
    if (th >= 1e-12) {
        a = sin(th) / th;
        b = (1.0 - cos(th)) / th2;
    }
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            const double KK = K[3 * r] * K[c] + K[3 * r + 1] * K[3 + c] + K[3 * r + 2] * K[6 + c];
            E[3 * r + c] = (r == c ? 1.0 : 0.0) + a * K[3 * r + c] + b * KK;
        }
}

// Fixed-order sum of the partials, then the Gauss-Newton update of the pose (one block).
__global__ __launch_bounds__(256) void k_gicp_solve(const double *__restrict__ partial, int nblocks,
                                                    double *__restrict__ pose, double *__restrict__ stats) {
    __shared__ double s[8][kGicpAcc];
    if (gicp_stopped(stats)) return;
    const int t = threadIdx.x;
    if (t < 8 * kGicpAcc) {
        const int e = t % kGicpAcc, g = t / kGicpAcc;
        double a = 0.0;
        for (int b = g; b < nblocks; b += 8) a += partial[(int64_t)b * kGicpAcc + e];
        s[g][e] = a;
    }
    __syncthreads();
    if (t < kGicpAcc) {
        double a = 0.0;
        for (int g = 0; g < 8; g++) a += s[g][t];
        stats[t] = a;
        s[0][t] = a;
    }
    __syncthreads();
    if (t != 0) return;
    stats[kStIters] += 1.0;
    if (s[0][kStCount] < 6.0) {
        stats[kStFailed] = 1.0;
        return;
    }
    double H[6][6], L[6][6] = {}, x[6];
    for (int a = 0; a < 6; a++)
        for (int b = a; b < 6; b++) H[a][b] = H[b][a] = s[0][tri(a, b)];
    // Cholesky H = L L^T, then L y = -g, L^T xi = y
    for (int c = 0; c < 6; c++) {
        double d = H[c][c];
        for (int k = 0; k < c; k++) d -= L[c][k] * L[c][k];
        if (!(d > 0.0)) {
            stats[kStFailed] = 1.0;
            return;
        }
        L[c][c] = sqrt(d);
        for (int r = c + 1; r < 6; r++) {
            double v = H[r][c];
            for (int k = 0; k < c; k++) v -= L[r][k] * L[c][k];
            L[r][c] = v / L[c][c];
        }
    }
    for (int r = 0; r < 6; r++) {
        double v = -s[0][21 + r];
        for (int k = 0; k < r; k++) v -= L[r][k] * x[k];
        x[r] = v / L[r][r];
    }
    for (int r = 5; r >= 0; r--) {
        double v = x[r];
        for (int k = r + 1; k < 6; k++) v -= L[k][r] * x[k];
        x[r] = v / L[r][r];
    }
    for (int e = 0; e < 6; e++) stats[kStXi + e] = x[e];
    double E[9], R[9], tt[3];
    so3_exp(x + 3, E);
    for (int e = 0; e < 9; e++) R[e] = pose[e];
    for (int e = 0; e < 3; e++) tt[e] = pose[9 + e];
    for (int r = 0; r < 3; r++) {
        for (int c = 0; c < 3; c++) pose[3 * r + c] = E[3 * r] * R[c] + E[3 * r + 1] * R[3 + c] + E[3 * r + 2] * R[6 + c];
        pose[9 + r] = E[3 * r] * tt[0] + E[3 * r + 1] * tt[1] + E[3 * r + 2] * tt[2] + x[r];
    }
    const double nr = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    const double np = sqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
    if (nr < kEpsRho && np < kEpsPhi) stats[kStConv] = 1.0;
}

size_t a256g(size_t b) { return (b + 255) & ~(size_t)255; }

struct GicpWs {
    double *src_cov, *tgt_cov, *partial;
    float4 *gp;
    uint32_t *f_src, *f_tgt, *off, *key, *val, *k2, *v2, *bucket;
    void *scan, *sort;
    size_t bytes;
};

int nblk256(int64_t n) { return (int)ceil_div(n > 0 ? n : 1, 256); }

GicpWs gicp_layout(void *base, int64_t n) {
    GicpWs w;
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t b) {
        void *r = p ? p + off : nullptr;
        off += a256g(b);
        return r;
    };
    const size_t nn = (size_t)(n > 0 ? n : 1);
    w.src_cov = (double *)take(6 * nn * 8);
    w.tgt_cov = (double *)take(6 * nn * 8);
    w.partial = (double *)take((size_t)nblk256(n) * kGicpAcc * 8);
    w.gp = (float4 *)take(nn * 16);
    w.f_src = (uint32_t *)take(nn * 4);
    w.f_tgt = (uint32_t *)take(nn * 4);
    w.off = (uint32_t *)take(nn * 4);
    w.key = (uint32_t *)take(nn * 4);
    w.val = (uint32_t *)take(nn * 4);
    w.k2 = (uint32_t *)take(nn * 4);
    w.v2 = (uint32_t *)take(nn * 4);
    w.bucket = (uint32_t *)take((size_t)(kBuckets + 1) * 4);
    w.scan = take(gsr_scan_ws_bytes(n));
    w.sort = take(gsr_sort_pairs_ws_bytes(n));
    w.bytes = off;
    return w;
}

double grid_cell(float d_corr) { return (double)d_corr * (1.0 + 1.0 / (1 << 20)); }

}  // namespace gsr

using namespace gsr;

extern "C" size_t gsr_gicp_ws_bytes(int64_t n) { return gicp_layout(nullptr, n).bytes; }

extern "C" gsr_status gsr_gicp_prepare_launch(const gsr_gaussians *g, const int32_t *seg, int32_t src_segment,
                                              const gsr_camera *cams, int n_cams, float d_max, float d_corr,
                                              uint32_t *src_index, uint32_t *tgt_index, uint32_t *counts,
                                              double *stats, void *ws, hipStream_t st) {
    const int64_t n = g->n;
    GicpWs w = gicp_layout(ws, n);
    gsr_status s = gsr_fill_u32_launch(stats, 0u, 2 * 40, st);
    if (s != GSR_OK) return s;
    if (n == 0) return gsr_fill_u32_launch(counts, 0u, 2, st);
    const double dd = (double)d_max * (double)d_max;
    k_gicp_flags<<<nblk256(n), 256, 0, st>>>(g->means, seg, n, src_segment, cams, n_cams, dd, w.f_src, w.f_tgt);
    s = gsr_scan_launch(w.f_src, n, w.off, counts, w.scan, st);
    if (s != GSR_OK) return s;
    k_gicp_compact<<<nblk256(n), 256, 0, st>>>(w.f_src, w.off, n, src_index);
    s = gsr_scan_launch(w.f_tgt, n, w.off, counts + 1, w.scan, st);
    if (s != GSR_OK) return s;
    k_gicp_compact<<<nblk256(n), 256, 0, st>>>(w.f_tgt, w.off, n, tgt_index);
    k_gicp_cov<<<nblk256(n), 256, 0, st>>>(src_index, counts, n, g->quats, g->log_scales, n, w.src_cov);
    k_gicp_cov<<<nblk256(n), 256, 0, st>>>(tgt_index, counts + 1, n, g->quats, g->log_scales, n, w.tgt_cov);
    s = gsr_grid_build_launch(g->means, n, tgt_index, counts + 1, n, grid_cell(d_corr), w.key, w.val, w.k2, w.v2,
                              w.bucket, w.sort, st);
    if (s != GSR_OK) return s;
    k_gicp_grid_points<<<nblk256(n), 256, 0, st>>>(g->means, n, tgt_index, counts, w.val, w.gp);
    return last_launch();
}

extern "C" gsr_status gsr_gicp_iterate_launch(const gsr_gaussians *g, const uint32_t *src_index,
                                              const uint32_t *tgt_index, const uint32_t *counts, float d_corr,
                                              double *pose, double *stats, int32_t *corr, int n_iter, void *ws,
                                              hipStream_t st) {
    const int64_t n = g->n;
    if (n == 0) return GSR_OK;
    GicpWs w = gicp_layout(ws, n);
    const double inv_cell = 1.0 / grid_cell(d_corr);
    const double dd = (double)d_corr * (double)d_corr;
    const int nb = nblk256(n);
    for (int it = 0; it < n_iter; it++) {
        k_gicp_linearise<<<nb, 256, 0, st>>>(g->means, n, src_index, tgt_index, counts, w.src_cov, w.tgt_cov, n, w.key,
                                             w.val, w.bucket, w.gp, inv_cell, dd, pose, stats, w.partial, corr);
        k_gicp_solve<<<1, 256, 0, st>>>(w.partial, nb, pose, stats);
    }
    return last_launch();
}

// ---- propagation of a corrected pose to a segment ------------------------------------------------
// The segment moves rigidly by (R, t): means R mu + t, orientations q_R (x) q (so R_q' = R R_q),
// and each SH degree l >= 1 turns with D_l, D_ab = integral of Y_a(d) Y_b(R^T d) over the sphere, so
// that the colour seen along R d afterwards is the colour seen along d before.  The integrand is
// a spherical polynomial of degree <= 6; the product rule of the 4-point Gauss-Legendre rule in
// z = cos(theta) with 8 equally spaced azimuths integrates it exactly.
namespace gsr {

constexpr int kShRotEntries = 9 + 25 + 49;  // D_1, D_2, D_3 row-major, then q_R (w, x, y, z)

// Real orthonormal SH without Condon-Shortley phase, degree <= 3, in float64 (index k = l^2 + l + m)
__device__ double sh_basis_d(int k, double x, double y, double z) {
    const double pi = 3.141592653589793;
    switch (k) {
        case 1: return sqrt(3.0 / (4.0 * pi)) * y;
        case 2: return sqrt(3.0 / (4.0 * pi)) * z;
        case 3: return sqrt(3.0 / (4.0 * pi)) * x;
        case 4: return sqrt(15.0 / (4.0 * pi)) * x * y;
        case 5: return sqrt(15.0 / (4.0 * pi)) * y * z;
        case 6: return sqrt(5.0 / (16.0 * pi)) * (3.0 * z * z - 1.0);
        case 7: return sqrt(15.0 / (4.0 * pi)) * x * z;
        case 8: return sqrt(15.0 / (16.0 * pi)) * (x * x - y * y);
        case 9: return sqrt(35.0 / (32.0 * pi)) * y * (3.0 * x * x - y * y);
        case 10: return sqrt(105.0 / (4.0 * pi)) * x * y * z;
        case 11: return sqrt(21.0 / (32.0 * pi)) * y * (5.0 * z * z - 1.0);
        case 12: return sqrt(7.0 / (16.0 * pi)) * z * (5.0 * z * z - 3.0);
        case 13: return sqrt(21.0 / (32.0 * pi)) * x * (5.0 * z * z - 1.0);
        case 14: return sqrt(105.0 / (16.0 * pi)) * z * (x * x - y * y);
        case 15: return sqrt(35.0 / (32.0 * pi)) * x * (x * x - 3.0 * y * y);
        default: return 0.28209479177387814;
    }
}

__global__ void k_sh_rotation(const double *__restrict__ pose, double *__restrict__ out) {
    const int e = threadIdx.x;
    double R[9];
    for (int i = 0; i < 9; i++) R[i] = pose[i];
    if (e < kShRotEntries) {
        int l, a, b;
        if (e < 9) l = 1, a = e / 3, b = e % 3;
        else if (e < 34) l = 2, a = (e - 9) / 5, b = (e - 9) % 5;
        else l = 3, a = (e - 34) / 7, b = (e - 34) % 7;
        const int ka = l * l + a, kb = l * l + b;
        // 4-point Gauss-Legendre nodes: roots of 35 z^4 - 30 z^2 + 3, weights 2 / ((1 - z^2) P4'(z)^2)
        const double r30 = sqrt(30.0);
        const double zs[2] = {sqrt((15.0 - 2.0 * r30) / 35.0), sqrt((15.0 + 2.0 * r30) / 35.0)};
        const double pi = 3.141592653589793;
        double acc = 0.0;
        for (int zi = 0; zi < 4; zi++) {
            const double z = zi < 2 ? zs[zi] : -zs[zi - 2];
            const double dp = (140.0 * z * z * z - 60.0 * z) / 8.0;  // P4'(z)
            const double wz = 2.0 / ((1.0 - z * z) * dp * dp);
            const double rho = sqrt(1.0 - z * z);
            for (int j = 0; j < 8; j++) {
                const double ph = 2.0 * pi * j / 8.0;
                const double x = rho * cos(ph), y = rho * sin(ph);
                // R^T d
                const double rx = R[0] * x + R[3] * y + R[6] * z;
                const double ry = R[1] * x + R[4] * y + R[7] * z;
                const double rz = R[2] * x + R[5] * y + R[8] * z;
                acc += wz * (2.0 * pi / 8.0) * sh_basis_d(ka, x, y, z) * sh_basis_d(kb, rx, ry, rz);
            }
        }
        out[e] = acc;
    } else if (e == kShRotEntries) {
        // q_R by Shepperd's method, sign with w >= 0
        double w, x, y, z;
        const double tr = R[0] + R[4] + R[8];
        if (tr > 0.0) {
            const double s = 2.0 * sqrt(tr + 1.0);
            w = 0.25 * s, x = (R[7] - R[5]) / s, y = (R[2] - R[6]) / s, z = (R[3] - R[1]) / s;
        } else if (R[0] > R[4] && R[0] > R[8]) {
            const double s = 2.0 * sqrt(1.0 + R[0] - R[4] - R[8]);
            w = (R[7] - R[5]) / s, x = 0.25 * s, y = (R[1] + R[3]) / s, z = (R[2] + R[6]) / s;
        } else if (R[4] > R[8]) {
            const double s = 2.0 * sqrt(1.0 + R[4] - R[0] - R[8]);
            w = (R[2] - R[6]) / s, x = (R[1] + R[3]) / s, y = 0.25 * s, z = (R[5] + R[7]) / s;
        } else {
            const double s = 2.0 * sqrt(1.0 + R[8] - R[0] - R[4]);
            w = (R[3] - R[1]) / s, x = (R[2] + R[6]) / s, y = (R[5] + R[7]) / s, z = 0.25 * s;
        }
        const double sg = w < 0.0 ? -1.0 : 1.0;
        out[kShRotEntries] = sg * w, out[kShRotEntries + 1] = sg * x;
        out[kShRotEntries + 2] = sg * y, out[kShRotEntries + 3] = sg * z;
    }
}

__global__ void k_transform_rows(float *__restrict__ means, float *__restrict__ quats, float *__restrict__ sh,
                                 int64_t n, int deg, const int32_t *__restrict__ seg, int32_t segment,
                                 const double *__restrict__ pose, const double *__restrict__ rot) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || seg[i] != segment) return;
    double R[9], t[3];
    for (int e = 0; e < 9; e++) R[e] = pose[e];
    for (int e = 0; e < 3; e++) t[e] = pose[9 + e];
    const double mx = means[i], my = means[n + i], mz = means[2 * n + i];
    means[i] = (float)(R[0] * mx + R[1] * my + R[2] * mz + t[0]);
    means[n + i] = (float)(R[3] * mx + R[4] * my + R[5] * mz + t[1]);
    means[2 * n + i] = (float)(R[6] * mx + R[7] * my + R[8] * mz + t[2]);
    const double aw = rot[kShRotEntries], ax = rot[kShRotEntries + 1], ay = rot[kShRotEntries + 2],
                 az = rot[kShRotEntries + 3];
    const double bw = quats[i], bx = quats[n + i], by = quats[2 * n + i], bz = quats[3 * n + i];
    quats[i] = (float)(aw * bw - ax * bx - ay * by - az * bz);
    quats[n + i] = (float)(aw * bx + ax * bw + ay * bz - az * by);
    quats[2 * n + i] = (float)(aw * by - ax * bz + ay * bw + az * bx);
    quats[3 * n + i] = (float)(aw * bz + ax * by - ay * bx + az * bw);
    int off = 0;
    for (int l = 1; l <= deg; l++) {
        const int w = 2 * l + 1;
        const double *D = rot + off;
        for (int ch = 0; ch < 3; ch++) {
            double c[7], o[7];
            for (int b = 0; b < w; b++) c[b] = sh[(int64_t)((l * l + b) * 3 + ch) * n + i];
            for (int a = 0; a < w; a++) {
                double v = 0.0;
                for (int b = 0; b < w; b++) v += D[a * w + b] * c[b];
                o[a] = v;
            }
            for (int a = 0; a < w; a++) sh[(int64_t)((l * l + a) * 3 + ch) * n + i] = (float)o[a];
        }
        off += w * w;
    }
}

// world -> camera of a moved segment: R_c R^T, t_c - R_c R^T t
__global__ void k_transform_cams(gsr_camera *__restrict__ cams, int n_cams, const uint8_t *__restrict__ mask,
                                 const double *__restrict__ pose) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_cams || (mask && !mask[k])) return;
    double R[9], t[3], Rc[9], tc[3], M[9];
    for (int e = 0; e < 9; e++) R[e] = pose[e], Rc[e] = cams[k].R[e];
    for (int e = 0; e < 3; e++) t[e] = pose[9 + e], tc[e] = cams[k].t[e];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) M[3 * a + b] = Rc[3 * a] * R[3 * b] + Rc[3 * a + 1] * R[3 * b + 1] + Rc[3 * a + 2] * R[3 * b + 2];
    for (int e = 0; e < 9; e++) cams[k].R[e] = (float)M[e];
    for (int a = 0; a < 3; a++) cams[k].t[a] = (float)(tc[a] - (M[3 * a] * t[0] + M[3 * a + 1] * t[1] + M[3 * a + 2] * t[2]));
}

}  // namespace gsr

extern "C" gsr_status gsr_transform_segment_launch(const gsr_params *p, int64_t n, int deg, const int32_t *seg,
                                                   int32_t segment, const double *pose, double *ws, hipStream_t st) {
    k_sh_rotation<<<1, 128, 0, st>>>(pose, ws);
    if (n > 0)
        k_transform_rows<<<(unsigned)ceil_div(n, 256), 256, 0, st>>>(p->means, p->quats, p->sh, n, deg, seg, segment,
                                                                     pose, ws);
    return last_launch();
}

extern "C" gsr_status gsr_transform_cameras_launch(gsr_camera *cams, int n_cams, const uint8_t *mask,
                                                   const double *pose, hipStream_t st) {
    if (n_cams > 0) k_transform_cams<<<(unsigned)ceil_div(n_cams, 64), 64, 0, st>>>(cams, n_cams, mask, pose);
    return last_launch();
}
