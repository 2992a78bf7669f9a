// Initialisation path: voxel-PCA geometric fitting (Sec. III-A, Eq. 1-2) and the cascaded
// Gaussian initialisation (Sec. III-B, Eq. 3, 5, 6).
//
// Voxel PCA: every point gets a packed 32-bit voxel key and a 64-bit SplitMix64 hash of
// (seed XOR index); three stable 32-bit radix sorts (hash low word, hash high word, key) group
// the points by voxel in ascending key order and, inside a voxel, by ascending hash.  A scan of
// the voxel heads numbers the voxels; one thread per voxel then fits its first (at most 32)
// points in double precision: mean, biased covariance, cyclic Jacobi eigensystem, canonical
// frame, planar / linear / unreliable class, and the trace of the descriptor's direction
// covariance, which Eq. 1-2 with isotropic point covariance sigma^2 I reduce to
// sigma^2 / N * sum_{m != k} (l_m + l_k) / (l_k - l_m)^2.  Given per-point world covariances,
// the same thread sums Eq. 2 itself, J_i Sigma_i J_i^T over the fitting points, for the full 6x6
// descriptor covariance and its trace.
#include "gsr_internal.h"

namespace gsr {

constexpr float kVoxel = 0.5f;
constexpr int kMaxPts = 32;
constexpr double kTauP = 2.5e-3, kTauL = 4.0, kLamFloor = 0.005 * 0.005, kSigma = 0.02, kRelTrace = 0.01;
constexpr int kMinPts = 5;
constexpr uint32_t kOutside = 0xffffffffu;

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// packed key: (kx + 1024) << 21 | (ky + 1024) << 10 | (kz + 511); kx, ky in [-1024, 1023],
// kz in [-511, 511] (so the all-ones word never names a voxel and marks points outside)
__global__ void k_vox_prep(const float *__restrict__ pts, int64_t n, uint64_t seed, uint32_t *__restrict__ key,
                           uint32_t *__restrict__ hlo, uint32_t *__restrict__ hhi, uint32_t *__restrict__ idx) {
    // hlo doubles as the first sort's key array
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float x = pts[i], y = pts[n + i], z = pts[2 * n + i];
        const float kxf = floorf(x / kVoxel), kyf = floorf(y / kVoxel), kzf = floorf(z / kVoxel);
        const bool in = kxf >= -1024.f && kxf <= 1023.f && kyf >= -1024.f && kyf <= 1023.f && kzf >= -511.f &&
                        kzf <= 511.f;
        key[i] = in ? ((uint32_t)((int)kxf + 1024) << 21) | ((uint32_t)((int)kyf + 1024) << 10) |
                          (uint32_t)((int)kzf + 511)
                    : kOutside;
        const uint64_t h = splitmix64(seed ^ (uint64_t)i);
        hlo[i] = (uint32_t)h;
        hhi[i] = (uint32_t)(h >> 32);
        idx[i] = (uint32_t)i;
    }
}

__global__ void k_gather_u32(const uint32_t *__restrict__ src, const uint32_t *__restrict__ idx, int64_t n,
                             uint32_t *__restrict__ dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[idx[i]];
}

__global__ void k_vox_heads(const uint32_t *__restrict__ skey, int64_t n, uint32_t *__restrict__ head) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        head[i] = (skey[i] != kOutside && (i == 0 || skey[i] != skey[i - 1])) ? 1u : 0u;
}

__global__ void k_vox_assign(const uint32_t *__restrict__ skey, const uint32_t *__restrict__ sidx,
                             const uint32_t *__restrict__ head, const uint32_t *__restrict__ hscan, int64_t n,
                             gsr_voxels V) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t p = sidx[i];
        V.point_order[i] = p;
        if (skey[i] == kOutside) {
            V.point_voxel[p] = kOutside;
            atomicAdd(V.n_outside, 1u);
            continue;
        }
        const uint32_t v = hscan[i] + head[i] - 1u;
        V.point_voxel[p] = v;
        if (head[i]) {
            V.start[v] = (uint32_t)i;
            V.key[v] = skey[i];
        }
    }
}

// 3x3 row-major products
__device__ __forceinline__ void mm3(const double *a, const double *b, double *c) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) c[i * 3 + j] = a[i * 3] * b[j] + a[i * 3 + 1] * b[3 + j] + a[i * 3 + 2] * b[6 + j];
}

// Cyclic Jacobi on a symmetric 3x3 (row-major a): plane rotations J over (0,1), (0,2), (1,2)
// that zero a_pq, a <- J^T a J, eigenvectors accumulated as the columns of w <- w J.
__device__ void jacobi3(double a[9], double w[9]) {
    for (int k = 0; k < 9; k++) w[k] = (k % 4 == 0) ? 1.0 : 0.0;
    const int pp[3] = {0, 0, 1}, qq[3] = {1, 2, 2};
    for (int sweep = 0; sweep < 60; sweep++) {
        const double off = a[1] * a[1] + a[2] * a[2] + a[5] * a[5];
        const double sc = a[0] * a[0] + a[4] * a[4] + a[8] * a[8];
        if (off <= 1e-30 * fmax(sc, 1e-300)) break;
        for (int r = 0; r < 3; r++) {
            const int p = pp[r], q = qq[r];
            const double apq = a[p * 3 + q];
            if (!(fabs(apq) > 1e-300)) continue;
            // tan(2 theta) = 2 a_pq / (a_qq - a_pp)
            const double th = 0.5 * atan2(2.0 * apq, a[q * 3 + q] - a[p * 3 + p]);
            const double c = cos(th), s = sin(th);
            double J[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, Jt[9], t[9];
            J[p * 3 + p] = c;
            J[q * 3 + q] = c;
            J[p * 3 + q] = s;
            J[q * 3 + p] = -s;
            for (int u = 0; u < 3; u++)
                for (int v = 0; v < 3; v++) Jt[u * 3 + v] = J[v * 3 + u];
            mm3(Jt, a, t);
            mm3(t, J, a);
            mm3(w, J, t);
            for (int k = 0; k < 9; k++) w[k] = t[k];
        }
    }
}

// COV: Eq. 1-2 with the per-point world covariances pcov [6][n] (xx, xy, xz, yy, yz, zz) instead
// of sigma^2 I; the full descriptor covariance goes to sg [21][n] (upper triangle, row-major)
// when sg is not null.
template <bool COV>
__global__ __launch_bounds__(256) void k_vox_pca(const float *__restrict__ pts, int64_t n, gsr_voxels V, const float *__restrict__ pcov,
                          float *__restrict__ sg) {
    const uint32_t nv = *V.n_voxels;
    const uint32_t nvalid = (uint32_t)n - *V.n_outside;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += gridDim.x * blockDim.x) {
        const uint32_t s0 = V.start[v];
        const uint32_t e0 = v + 1 < nv ? V.start[v + 1] : nvalid;
        const uint32_t cnt = e0 - s0;
        const int m = cnt < (uint32_t)kMaxPts ? (int)cnt : kMaxPts;
        V.count[v] = cnt;
        double mu[3] = {0, 0, 0};
        for (int j = 0; j < m; j++) {
            const uint32_t p = V.point_order[s0 + j];
            mu[0] += pts[p];
            mu[1] += pts[n + p];
            mu[2] += pts[2 * n + p];
        }
        for (int c = 0; c < 3; c++) mu[c] /= m;
        double C[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int j = 0; j < m; j++) {
            const uint32_t p = V.point_order[s0 + j];
            const double d[3] = {pts[p] - mu[0], pts[n + p] - mu[1], pts[2 * n + p] - mu[2]};
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) C[a * 3 + b] += d[a] * d[b];
        }
        for (int k = 0; k < 9; k++) C[k] /= m;
        double A[9], W[9];
        for (int k = 0; k < 9; k++) A[k] = C[k];
        jacobi3(A, W);
        // ascending eigenvalues (stable order on ties), eigenvectors as W's columns
        double lam[3] = {A[0], A[4], A[8]};
        int ord[3] = {0, 1, 2};
        for (int i = 1; i < 3; i++)
            for (int j = i; j > 0 && lam[ord[j]] < lam[ord[j - 1]]; j--) {
                const int t = ord[j];
                ord[j] = ord[j - 1];
                ord[j - 1] = t;
            }
        const double l[3] = {lam[ord[0]], lam[ord[1]], lam[ord[2]]};
        // R_pca columns (v_max, v_mid, v_min): largest |component| positive, then det = +1
        double R[9];
        for (int c = 0; c < 3; c++) {
            const int src = ord[2 - c];
            int big = 0;
            for (int r = 1; r < 3; r++)
                if (fabs(W[r * 3 + src]) > fabs(W[big * 3 + src])) big = r;
            const double sg = W[big * 3 + src] < 0 ? -1.0 : 1.0;
            for (int r = 0; r < 3; r++) R[r * 3 + c] = sg * W[r * 3 + src];
        }
        const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                           R[2] * (R[3] * R[7] - R[4] * R[6]);
        if (det < 0)
            for (int r = 0; r < 3; r++) R[r * 3 + 2] = -R[r * 3 + 2];
        uint8_t cls = 2;
        if (l[0] < kTauP) cls = 0;
        else if (l[2] / l[0] > kTauL) cls = 1;
        if (m < kMinPts) cls = 2;
        double tr = INFINITY;
        if (cls != 2 && !COV) {
            const int k = cls == 0 ? 0 : 2;
            double t = 0.0;
            for (int q = 0; q < 3; q++)
                if (q != k) t += (l[q] + l[k]) / ((l[k] - l[q]) * (l[k] - l[q]));
            tr = kSigma * kSigma / m * t;
        }
        if (COV) {
            double G[21];
#pragma unroll
            for (int e = 0; e < 21; e++) G[e] = 0.0;
            if (cls != 2) {
                // eigenvectors ascending (v_min, v_mid, v_max) = R_pca columns 2, 1, 0
                const int k = cls == 0 ? 0 : 2;
                double ev[3][3];
#pragma unroll
                for (int q = 0; q < 3; q++)
#pragma unroll
                    for (int r = 0; r < 3; r++) ev[q][r] = R[r * 3 + (2 - q)];
                double vk[3], lk = k == 0 ? l[0] : l[2];
#pragma unroll
                for (int r = 0; r < 3; r++) vk[r] = k == 0 ? ev[0][r] : ev[2][r];
                for (int j = 0; j < m; j++) {
                    const uint32_t p = V.point_order[s0 + j];
                    const double d[3] = {pts[p] - mu[0], pts[n + p] - mu[1], pts[2 * n + p] - mu[2]};
                    const double dk = d[0] * vk[0] + d[1] * vk[1] + d[2] * vk[2];
                    // T = V F = sum_{q != k} v_q f_q^T, f_q = ((d.v_q) v_k + (d.v_k) v_q) / (m (l_k - l_q))
                    double T[9];
#pragma unroll
                    for (int e = 0; e < 9; e++) T[e] = 0.0;
#pragma unroll
                    for (int q = 0; q < 3; q++) {
                        if (q == k) continue;
                        const double dq = d[0] * ev[q][0] + d[1] * ev[q][1] + d[2] * ev[q][2];
                        const double inv = 1.0 / (m * (lk - l[q]));
#pragma unroll
                        for (int r = 0; r < 3; r++)
#pragma unroll
                            for (int c = 0; c < 3; c++) T[r * 3 + c] += ev[q][r] * ((dq * vk[c] + dk * ev[q][c]) * inv);
                    }
                    const double S[9] = {pcov[p],         pcov[n + p],     pcov[2 * n + p],
                                         pcov[n + p],     pcov[3 * n + p], pcov[4 * n + p],
                                         pcov[2 * n + p], pcov[4 * n + p], pcov[5 * n + p]};
                    // J = [T; I/m] (6 x 3), G += J S J^T
                    double J[6][3], JS[6][3];
#pragma unroll
                    for (int r = 0; r < 3; r++)
#pragma unroll
                        for (int c = 0; c < 3; c++) J[r][c] = T[r * 3 + c], J[3 + r][c] = r == c ? 1.0 / m : 0.0;
#pragma unroll
                    for (int r = 0; r < 6; r++)
#pragma unroll
                        for (int c = 0; c < 3; c++) JS[r][c] = J[r][0] * S[c] + J[r][1] * S[3 + c] + J[r][2] * S[6 + c];
#pragma unroll
                    for (int r = 0; r < 6; r++)
#pragma unroll
                        for (int c = r; c < 6; c++)
                            G[r * 6 - r * (r - 1) / 2 + (c - r)] += JS[r][0] * J[c][0] + JS[r][1] * J[c][1] + JS[r][2] * J[c][2];
                }
                tr = G[0] + G[6] + G[11];  // (0,0), (1,1), (2,2) of the upper triangle
            }
            if (sg)
#pragma unroll
                for (int e = 0; e < 21; e++) sg[(int64_t)e * n + v] = (float)G[e];
        }
        const int64_t N = n;
        for (int c = 0; c < 3; c++) {
            V.mu[c * N + v] = (float)mu[c];
            V.evals[c * N + v] = (float)l[c];
            V.s_pca[c * N + v] = (float)(0.5 * log(fmax(l[2 - c], kLamFloor)));
        }
        for (int k = 0; k < 9; k++) V.R[k * N + v] = (float)R[k];
        V.trace[v] = (float)tr;
        V.cls[v] = cls;
        V.reliable[v] = (cls != 2 && tr < kRelTrace) ? 1 : 0;
    }
}

}  // namespace gsr

using namespace gsr;

extern "C" gsr_status gsr_scan_launch(const uint32_t *, int64_t, uint32_t *, uint32_t *, void *, hipStream_t);
extern "C" size_t gsr_scan_ws_bytes(int64_t n);
extern "C" size_t gsr_sort_pairs_ws_bytes(int64_t n);
extern "C" gsr_status gsr_sort_pairs_launch(uint32_t *, uint32_t *, uint32_t *, uint32_t *, uint32_t, int, void *,
                                            hipStream_t);
extern "C" gsr_status gsr_fill_u32_launch(void *, uint32_t, int64_t, hipStream_t);

namespace {
struct VoxWs {
    uint32_t *key, *hhi, *k0, *v0, *k1, *v1, *head, *hscan;
    void *sort_ws, *scan_ws;
    size_t bytes;
};
size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
VoxWs vox_layout(void *base, int64_t n) {
    VoxWs w{};
    char *p = static_cast<char *>(base);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        void *r = p ? p + off : nullptr;
        off += al256(bytes);
        return r;
    };
    const size_t nb = (size_t)(n > 0 ? n : 1) * 4;
    w.key = (uint32_t *)take(nb);
    w.hhi = (uint32_t *)take(nb);
    w.k0 = (uint32_t *)take(nb);
    w.v0 = (uint32_t *)take(nb);
    w.k1 = (uint32_t *)take(nb);
    w.v1 = (uint32_t *)take(nb);
    w.head = (uint32_t *)take(nb);
    w.hscan = (uint32_t *)take(nb);
    w.sort_ws = take(gsr_sort_pairs_ws_bytes(n));
    w.scan_ws = take(gsr_scan_ws_bytes(n));
    w.bytes = off;
    return w;
}
int grid(int64_t n) { return (int)(ceil_div(n > 0 ? n : 1, 256) < 16384 ? ceil_div(n > 0 ? n : 1, 256) : 16384); }
}  // namespace

extern "C" size_t gsr_voxel_pca_ws_bytes(int64_t n) { return vox_layout(nullptr, n).bytes; }

static gsr_status voxel_pca_run(const float *pts, int64_t n, uint64_t seed, const gsr_voxels *out, void *ws,
                                hipStream_t st, const float *pcov, float *sg) {
    gsr_status s = gsr_fill_u32_launch(out->n_outside, 0u, 1, st);
    if (s != GSR_OK) return s;
    if (n == 0) return gsr_fill_u32_launch(out->n_voxels, 0u, 1, st);
    VoxWs w = vox_layout(ws, n);
    const int g = grid(n);
    k_vox_prep<<<g, 256, 0, st>>>(pts, n, seed, w.key, w.k0, w.hhi, w.v0);
    // (hash low, hash high, voxel key): three stable sorts, least significant first; each of
    // 4 passes, so the result lands back in (k0, v0)
    s = gsr_sort_pairs_launch(w.k0, w.v0, w.k1, w.v1, (uint32_t)n, 32, w.sort_ws, st);
    if (s != GSR_OK) return s;
    k_gather_u32<<<g, 256, 0, st>>>(w.hhi, w.v0, n, w.k0);
    s = gsr_sort_pairs_launch(w.k0, w.v0, w.k1, w.v1, (uint32_t)n, 32, w.sort_ws, st);
    if (s != GSR_OK) return s;
    k_gather_u32<<<g, 256, 0, st>>>(w.key, w.v0, n, w.k0);
    s = gsr_sort_pairs_launch(w.k0, w.v0, w.k1, w.v1, (uint32_t)n, 32, w.sort_ws, st);
    if (s != GSR_OK) return s;
    k_vox_heads<<<g, 256, 0, st>>>(w.k0, n, w.head);
    s = gsr_scan_launch(w.head, n, w.hscan, out->n_voxels, w.scan_ws, st);
    if (s != GSR_OK) return s;
    k_vox_assign<<<g, 256, 0, st>>>(w.k0, w.v0, w.head, w.hscan, n, *out);
    if (pcov) k_vox_pca<true><<<g, 256, 0, st>>>(pts, n, *out, pcov, sg);
    else k_vox_pca<false><<<g, 256, 0, st>>>(pts, n, *out, nullptr, nullptr);
    return last_launch();
}

extern "C" gsr_status gsr_voxel_pca_launch(const float *pts, int64_t n, uint64_t seed, const gsr_voxels *out,
                                           void *ws, hipStream_t st) {
    return voxel_pca_run(pts, n, seed, out, ws, st, nullptr, nullptr);
}

extern "C" gsr_status gsr_voxel_pca_cov_launch(const float *pts, const float *pcov, int64_t n, uint64_t seed,
                                               const gsr_voxels *out, float *sg, void *ws, hipStream_t st) {
    return voxel_pca_run(pts, n, seed, out, ws, st, pcov, sg);
}

// ---- cascaded initialisation (Eq. 3, 5, 6) ------------------------------------------------------
namespace gsr {

constexpr float kOpacityConst = 0.1f;
constexpr float kY00 = 0.28209479177387814f;

// Eq. 3's valid model prediction: finite outputs, non-zero quaternion, log-scales in
// [log 2 mm, log 0.5 m].  pred [8][stride] = (s[3], q[4], omega) per voxel.
__device__ __forceinline__ bool pred_valid(const float *pred, int64_t stride, uint32_t v) {
    if (!pred) return false;
    float q2 = 0.f;
    for (int k = 0; k < 8; k++) {
        const float x = pred[k * stride + v];
        if (!isfinite(x)) return false;
        if (k >= 3 && k < 7) q2 += x * x;
    }
    if (!(q2 > 0.f)) return false;
    for (int k = 0; k < 3; k++) {
        const float s = pred[k * stride + v];
        if (s < -6.2146080984221914f || s > -0.69314718055994531f) return false;  // log 0.002, log 0.5
    }
    return true;
}

// Per-segment point counts for beta.  Points of one segment arrive together, so per-point global
// atomics would all hit one address; each workgroup counts in LDS (up to kSegLds segments) and
// adds its totals once.
constexpr int kSegLds = 1024;

__global__ __launch_bounds__(256) void k_seg_counts(const uint32_t *__restrict__ pvox,
                                                    const uint8_t *__restrict__ reliable, const float *__restrict__ pred,
                                                    int64_t n, const int32_t *__restrict__ seg, int nseg,
                                                    uint32_t *__restrict__ cnt, uint32_t *__restrict__ fb) {
    __shared__ uint32_t s_cnt[kSegLds], s_fb[kSegLds];
    const bool lds = nseg <= kSegLds;
    if (lds)
        for (int e = threadIdx.x; e < nseg; e += 256) s_cnt[e] = s_fb[e] = 0u;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = pvox[i];
        const int s = seg ? seg[i] : 0;
        if (v == kOutside || s < 0 || s >= nseg) continue;
        const bool f = reliable[v] && !pred_valid(pred, n, v);
        if (lds) {
            atomicAdd(&s_cnt[s], 1u);
            if (f) atomicAdd(&s_fb[s], 1u);
        } else {
            atomicAdd(&cnt[s], 1u);
            if (f) atomicAdd(&fb[s], 1u);
        }
    }
    __syncthreads();
    if (lds)
        for (int e = threadIdx.x; e < nseg; e += 256) {
            if (s_cnt[e]) atomicAdd(&cnt[e], s_cnt[e]);
            if (s_fb[e]) atomicAdd(&fb[e], s_fb[e]);
        }
}

// rotation matrix (row-major) -> unit quaternion (w, x, y, z), w >= 0, largest-pivot method
__device__ void rot_to_quat(const double r[9], double q[4]) {
    const double tr = r[0] + r[4] + r[8];
    if (tr > 0) {
        const double s = 2.0 * sqrt(1.0 + tr);
        q[0] = 0.25 * s, q[1] = (r[7] - r[5]) / s, q[2] = (r[2] - r[6]) / s, q[3] = (r[3] - r[1]) / s;
    } else if (r[0] > r[4] && r[0] > r[8]) {
        const double s = 2.0 * sqrt(1.0 + r[0] - r[4] - r[8]);
        q[0] = (r[7] - r[5]) / s, q[1] = 0.25 * s, q[2] = (r[1] + r[3]) / s, q[3] = (r[2] + r[6]) / s;
    } else if (r[4] > r[8]) {
        const double s = 2.0 * sqrt(1.0 + r[4] - r[0] - r[8]);
        q[0] = (r[2] - r[6]) / s, q[1] = (r[1] + r[3]) / s, q[2] = 0.25 * s, q[3] = (r[5] + r[7]) / s;
    } else {
        const double s = 2.0 * sqrt(1.0 + r[8] - r[0] - r[4]);
        q[0] = (r[3] - r[1]) / s, q[1] = (r[2] + r[6]) / s, q[2] = (r[5] + r[7]) / s, q[3] = 0.25 * s;
    }
    const double nq = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double sg = q[0] < 0 ? -1.0 : 1.0;
    for (int k = 0; k < 4; k++) q[k] = sg * q[k] / nq;
}

__global__ void k_cascade(const float *__restrict__ pts, const float *__restrict__ col, const float *__restrict__ depth,
                          const int32_t *__restrict__ seg, int nseg, int64_t n, gsr_voxels V,
                          const float *__restrict__ pred, float focal, float beta_fixed,
                          const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ fb, int K, gsr_params out,
                          uint8_t *__restrict__ branch, int anchored) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t v = V.point_voxel[i];
        for (int c = 0; c < 3; c++) {
            out.means[c * n + i] = pts[c * n + i];
            out.sh[c * n + i] = (col[c * n + i] - 0.5f) / kY00;
        }
        for (int k = 3; k < 3 * K; k++) out.sh[k * n + i] = 0.f;
        const bool inside = v != kOutside;
        const bool valid = inside && pred_valid(pred, n, v);
        const bool rel = inside && V.reliable[v];
        const uint8_t br = valid ? 0 : (rel ? 1 : 2);
        branch[i] = br;
        float ls[3], q[4], lo = logf(kOpacityConst / (1.f - kOpacityConst));
        if (br == 0) {
            float nq = 0.f;
            for (int k = 0; k < 4; k++) nq += pred[(3 + k) * n + v] * pred[(3 + k) * n + v];
            nq = sqrtf(nq);
            for (int k = 0; k < 3; k++) ls[k] = pred[k * n + v];
            if (anchored) {
                // Eq. 4: keep the axis ratios a = exp(s - max s) and anchor the size at d / f
                const float mx = fmaxf(ls[0], fmaxf(ls[1], ls[2]));
                const float a0 = logf(depth[i] / focal);
                for (int k = 0; k < 3; k++) ls[k] = a0 + (ls[k] - mx);
            }
            for (int k = 0; k < 4; k++) q[k] = pred[(3 + k) * n + v] / nq;
            lo = pred[7 * n + v];
        } else if (br == 1) {
            float beta = beta_fixed;
            if (!(beta > 0.f)) {
                const int s = seg ? seg[i] : 0;
                const uint32_t c = (s >= 0 && s < nseg) ? cnt[s] : 0u;
                const float rho = c ? (float)fb[s] / (float)c : 0.f;
                beta = fminf(fmaxf(1.f - rho, 0.5f), 1.f);
            }
            const float lb = logf(beta);
            for (int k = 0; k < 3; k++) ls[k] = V.s_pca[k * n + v] + lb;
            double r[9], qd[4];
            for (int k = 0; k < 9; k++) r[k] = V.R[k * n + v];
            rot_to_quat(r, qd);
            for (int k = 0; k < 4; k++) q[k] = (float)qd[k];
        } else {
            const float s = logf(depth[i] / focal);
            ls[0] = ls[1] = ls[2] = s;
            q[0] = 1.f, q[1] = q[2] = q[3] = 0.f;
        }
        for (int k = 0; k < 3; k++) out.log_scales[k * n + i] = ls[k];
        for (int k = 0; k < 4; k++) out.quats[k * n + i] = q[k];
        out.opacity_logits[i] = lo;
    }
}

// Training targets of the point network (Sec. III-B): for every voxel, the mean covariance
// R(q/|q|) diag(exp(2 s)) R^T (xx, xy, xz, yy, yz, zz) and the mean opacity sigmoid(logit) of the
// Gaussians seeded one per point, over all the voxel's points.  One thread per voxel sums in float64
// in the voxel's point order (fixed, so the targets repeat exactly); rows at or past the voxel count
// are zero with has = 0.
__global__ void k_voxel_targets(const float *__restrict__ ls, const float *__restrict__ qs,
                                const float *__restrict__ lo, int64_t n, gsr_voxels V, float *__restrict__ cov,
                                float *__restrict__ ot, uint8_t *__restrict__ has) {
    const uint32_t nv = *V.n_voxels;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, op = 0.0;
        const uint32_t c = v < nv ? V.count[v] : 0u;
        const uint32_t s0 = c ? V.start[v] : 0u;
        for (uint32_t k = 0; k < c; k++) {
            const int64_t i = V.point_order[s0 + k];
            double w = qs[i], x = qs[n + i], y = qs[2 * n + i], z = qs[3 * n + i];
            const double nq = sqrt(w * w + x * x + y * y + z * z);
            w /= nq, x /= nq, y /= nq, z /= nq;
            const double R[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                                    {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                                    {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
            const double e[3] = {exp(2.0 * (double)ls[i]), exp(2.0 * (double)ls[n + i]), exp(2.0 * (double)ls[2 * n + i])};
            int q = 0;
            for (int a = 0; a < 3; a++)
                for (int b = a; b < 3; b++, q++)
                    acc[q] += R[a][0] * e[0] * R[b][0] + R[a][1] * e[1] * R[b][1] + R[a][2] * e[2] * R[b][2];
            op += 1.0 / (1.0 + exp(-(double)lo[i]));
        }
        const double inv = c ? 1.0 / (double)c : 0.0;
        for (int q = 0; q < 6; q++) cov[q * n + v] = (float)(acc[q] * inv);
        ot[v] = (float)(op * inv);
        has[v] = c ? 1 : 0;
    }
}


}  // namespace gsr

extern "C" size_t gsr_cascade_ws_bytes(int nseg) { return (size_t)(2 * (nseg > 0 ? nseg : 1) * 4 + 512); }

extern "C" gsr_status gsr_cascade_launch(const float *pts, const float *col, const float *depth, const int32_t *seg,
                                         int nseg, int64_t n, const gsr_voxels *vox, const float *pred, float focal,
                                         float beta, int sh_degree, const gsr_params *out, uint8_t *branch, void *ws,
                                         hipStream_t st, int anchored) {
    if (n == 0) return GSR_OK;
    uint32_t *cnt = static_cast<uint32_t *>(ws);
    uint32_t *fb = cnt + (nseg > 0 ? nseg : 1);
    gsr_status s = gsr_fill_u32_launch(cnt, 0u, 2 * (int64_t)(nseg > 0 ? nseg : 1), st);
    if (s != GSR_OK) return s;
    const int g = grid(n);
    k_seg_counts<<<g < 1024 ? g : 1024, 256, 0, st>>>(vox->point_voxel, vox->reliable, pred, n, seg, nseg, cnt, fb);
    k_cascade<<<g, 256, 0, st>>>(pts, col, depth, seg, nseg, n, *vox, pred, focal, beta, cnt, fb,
                                 (sh_degree + 1) * (sh_degree + 1), *out, branch, anchored);
    return last_launch();
}

extern "C" gsr_status gsr_voxel_targets_launch(const gsr_params *g, int64_t n, const gsr_voxels *vox, float *cov,
                                              float *ot, uint8_t *has, hipStream_t st) {
    if (n == 0) return GSR_OK;
    const int64_t nb = ceil_div(n, 256);
    k_voxel_targets<<<(int)(nb < 4096 ? nb : 4096), 256, 0, st>>>(g->log_scales, g->quats, g->opacity_logits, n,
                                                                   *vox, cov, ot, has);
    return last_launch();
}
