"""FP64 oracle of the initialisation path: voxel-PCA geometric fitting (paper Sec. III-A, Eq. 1-2)
and the cascaded Gaussian initialisation (Sec. III-B, Eq. 3, 5, 6).

TEST INFRASTRUCTURE ONLY: imported by the tests and the benchmark's CPU leg, never by the
product path, and sharing no code with it.  Plain numpy in double precision; every step follows
the definition it cites, vectorised over voxels but without any blocking or reordering.

Readings where the paper prints no value (kept identical on the GPU side):
  voxel edge 0.5 m on a flat grid; at most 32 points per voxel, the ones with the smallest
  SplitMix64(seed XOR point index); biased covariance; eigenvalues ascending; an eigenvector's
  largest-magnitude component is positive, then v_min flips so that det[v_max v_mid v_min] = +1;
  planar if lambda_min < tau_p = 2.5e-3 m^2, else linear if lambda_max / lambda_min > tau_l = 4,
  else unreliable (also unreliable below 5 points); s_pca = 0.5 log max(lambda, (5 mm)^2) in the
  column order (v_max, v_mid, v_min); reliable iff planar or linear and the trace of the
  direction block of the descriptor covariance (Eq. 1-2 with every point covariance sigma^2 I,
  sigma = 2 cm) is below 0.1^2; non-model branches get opacity 0.1 and zero higher-order SH.
"""
from __future__ import annotations

import numpy as np

VOXEL = 0.5
MAX_PTS = 32
TAU_P = 2.5e-3
TAU_L = 4.0
LAMBDA_FLOOR = 0.005 ** 2
MIN_PTS = 5
SIGMA_PT = 0.02
REL_TRACE = 0.1 ** 2
OPACITY_CONST = 0.1
LOG_S_MIN, LOG_S_MAX = np.log(0.002), np.log(0.5)
Y00 = 0.28209479177387814  # 1 / (2 sqrt(pi))

PLANAR, LINEAR, UNRELIABLE = 0, 1, 2
MASK64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output function (Steele, Lea and Flood, 2014) of 64-bit inputs, as uint64."""
    z = (np.asarray(x, np.uint64) + np.uint64(0x9E3779B97F4A7C15))
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def voxel_keys(points):
    """Integer voxel coordinates floor(p / 0.5 m), shape [N, 3]."""
    return np.floor(np.asarray(points, np.float64) / VOXEL).astype(np.int64)


def jacobi_eigh3(C, sweeps=60):
    """Cyclic Jacobi eigen-decomposition of symmetric 3x3 matrices C [n, 3, 3]: plane rotations
    that zero one off-diagonal entry at a time.  Returns eigenvalues ascending [n, 3] and the
    eigenvectors as columns [n, 3, 3] in the same order."""
    A = np.array(C, np.float64, copy=True)
    n = A.shape[0]
    V = np.broadcast_to(np.eye(3), (n, 3, 3)).copy()
    for _ in range(sweeps):
        off = A[:, 0, 1] ** 2 + A[:, 0, 2] ** 2 + A[:, 1, 2] ** 2
        scale = np.einsum("nii->n", A * A)
        if np.all(off <= 1e-30 * np.maximum(scale, 1e-300)):
            break
        for p, q in ((0, 1), (0, 2), (1, 2)):
            apq = A[:, p, q]
            app, aqq = A[:, p, p], A[:, q, q]
            act = np.abs(apq) > 1e-300
            # rotation angle that annihilates A[p, q]: tan(2 theta) = 2 a_pq / (a_qq - a_pp)
            theta = np.where(act, 0.5 * np.arctan2(2.0 * apq, aqq - app), 0.0)
            c, s = np.cos(theta), np.sin(theta)
            Jm = np.broadcast_to(np.eye(3), (n, 3, 3)).copy()
            Jm[:, p, p] = c
            Jm[:, q, q] = c
            Jm[:, p, q] = s
            Jm[:, q, p] = -s
            A = np.einsum("nji,njk,nkl->nil", Jm, A, Jm)
            V = np.einsum("nij,njk->nik", V, Jm)
    w = np.stack([A[:, 0, 0], A[:, 1, 1], A[:, 2, 2]], axis=1)
    order = np.argsort(w, axis=1, kind="stable")
    w = np.take_along_axis(w, order, axis=1)
    V = np.take_along_axis(V, order[:, None, :], axis=2)
    return w, V


def canonical_frame(V):
    """Columns (v_min, v_mid, v_max) -> R_pca = [v_max v_mid v_min] with each vector's largest
    |component| positive, then v_min flipped so that det R_pca = +1."""
    R = V[:, :, ::-1].copy()
    for j in range(3):
        col = R[:, :, j]
        big = np.take_along_axis(col, np.argmax(np.abs(col), axis=1)[:, None], axis=1)[:, 0]
        R[:, :, j] *= np.where(big < 0, -1.0, 1.0)[:, None]
    det = np.linalg.det(R)
    R[:, :, 2] *= np.where(det < 0, -1.0, 1.0)[:, None]
    return R


def direction_trace_points(d, lam, k):
    """Eq. 1-2: J_i's direction rows are V F_i with f_i^(m) = d_i^T (v_m v_k^T + v_k v_m^T) /
    (N (lambda_k - lambda_m)) for m != k; Sigma_g,dir = sum_i V F_i (sigma^2 I) F_i^T V^T.  d [N, 3]
    are the centred points in the eigenbasis, so v_m is the m-th unit vector."""
    N = d.shape[0]
    tr = 0.0
    for i in range(N):
        F = np.zeros((3, 3))
        for m in range(3):
            if m == k:
                continue
            vm, vk = np.eye(3)[m], np.eye(3)[k]
            F[m] = d[i] @ (np.outer(vm, vk) + np.outer(vk, vm)) / (N * (lam[k] - lam[m]))
        tr += SIGMA_PT ** 2 * np.trace(F @ F.T)
    return tr


def voxel_pca(points, seed):
    """Voxel-PCA fitting of a point cloud (Sec. III-A).  Voxels in ascending (kx, ky, kz) order.

    Returns dict with per voxel: key [V, 3], n_all, n (selected), ids (list of selected point
    indices, ascending hash), mu [V, 3], C [V, 3, 3], evals [V, 3] ascending, R [V, 3, 3]
    (= [v_max v_mid v_min]), s_pca [V, 3] (column order of R), cls, trace, reliable; and per point
    voxel [N] (index of its voxel)."""
    P = np.asarray(points, np.float64)
    N = P.shape[0]
    key = voxel_keys(P)
    h = splitmix64(np.uint64(seed) ^ np.arange(N, dtype=np.uint64))
    # group by voxel (lexicographic key), inside a voxel by ascending hash, then index
    order = np.lexsort((np.arange(N), h, key[:, 2], key[:, 1], key[:, 0]))
    ks = key[order]
    start = np.concatenate([[0], np.nonzero(np.any(ks[1:] != ks[:-1], axis=1))[0] + 1, [N]])
    nv = len(start) - 1
    voxel = np.empty(N, np.int64)
    ids, n_all = [], np.diff(start)
    for v in range(nv):
        members = order[start[v]:start[v + 1]]
        voxel[members] = v
        ids.append(members[:MAX_PTS])
    n = np.array([len(x) for x in ids])
    mu = np.stack([P[x].mean(axis=0) for x in ids])
    C = np.stack([(P[x] - mu[v]).T @ (P[x] - mu[v]) / len(x) for v, x in enumerate(ids)])
    lam, V = jacobi_eigh3(C)
    R = canonical_frame(V)
    cls = np.full(nv, UNRELIABLE)
    lmin, lmax = lam[:, 0], lam[:, 2]
    planar = lmin < TAU_P
    with np.errstate(divide="ignore", invalid="ignore"):
        linear = ~planar & (lmax / lmin > TAU_L)
    cls[planar] = PLANAR
    cls[linear] = LINEAR
    cls[n < MIN_PTS] = UNRELIABLE
    trace = np.full(nv, np.inf)
    for v in range(nv):
        if cls[v] == UNRELIABLE:
            continue
        k = 0 if cls[v] == PLANAR else 2
        d = (P[ids[v]] - mu[v]) @ V[v]  # coordinates in the eigenbasis (v_min, v_mid, v_max)
        trace[v] = direction_trace_points(d, lam[v], k)
    reliable = (cls != UNRELIABLE) & (trace < REL_TRACE)
    s_pca = 0.5 * np.log(np.maximum(lam[:, ::-1], LAMBDA_FLOOR))
    return dict(key=ks[start[:-1]], n_all=n_all, n=n, ids=ids, mu=mu, C=C, evals=lam, R=R, s_pca=s_pca,
                cls=cls, trace=trace, reliable=reliable, voxel=voxel)


def rot_to_quat(R):
    """Rotation matrices [n, 3, 3] -> unit quaternions (w, x, y, z) with w >= 0 (largest-pivot
    method)."""
    n = R.shape[0]
    q = np.zeros((n, 4))
    tr = R[:, 0, 0] + R[:, 1, 1] + R[:, 2, 2]
    for i in range(n):
        r = R[i]
        if tr[i] > 0:
            s = 2.0 * np.sqrt(1.0 + tr[i])
            q[i] = [0.25 * s, (r[2, 1] - r[1, 2]) / s, (r[0, 2] - r[2, 0]) / s, (r[1, 0] - r[0, 1]) / s]
        elif r[0, 0] > r[1, 1] and r[0, 0] > r[2, 2]:
            s = 2.0 * np.sqrt(1.0 + r[0, 0] - r[1, 1] - r[2, 2])
            q[i] = [(r[2, 1] - r[1, 2]) / s, 0.25 * s, (r[0, 1] + r[1, 0]) / s, (r[0, 2] + r[2, 0]) / s]
        elif r[1, 1] > r[2, 2]:
            s = 2.0 * np.sqrt(1.0 + r[1, 1] - r[0, 0] - r[2, 2])
            q[i] = [(r[0, 2] - r[2, 0]) / s, (r[0, 1] + r[1, 0]) / s, 0.25 * s, (r[1, 2] + r[2, 1]) / s]
        else:
            s = 2.0 * np.sqrt(1.0 + r[2, 2] - r[0, 0] - r[1, 1])
            q[i] = [(r[1, 0] - r[0, 1]) / s, (r[0, 2] + r[2, 0]) / s, (r[1, 2] + r[2, 1]) / s, 0.25 * s]
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q *= np.where(q[:, :1] < 0, -1.0, 1.0)
    return q


def prediction_valid(pred):
    """Eq. 3's "valid model prediction": every output finite and each log-scale within
    [log 2 mm, log 0.5 m].  pred [V, 8] = (s[3], q[4], omega).  The network's outputs are float32,
    so the bound test is taken in float32: both the log-scale and the two bounds are rounded to
    float32 before comparing (inclusive at both ends)."""
    pred = np.asarray(pred, np.float64)
    fin = np.all(np.isfinite(pred), axis=1) & (np.linalg.norm(pred[:, 3:7], axis=1) > 0)
    s = pred[:, :3].astype(np.float32)
    return fin & np.all((s >= np.float32(LOG_S_MIN)) & (s <= np.float32(LOG_S_MAX)), axis=1)


def cascade(points, colors, depth, segment, vox, pred=None, f=640.0, beta=None, sh_degree=0, anchored=False):
    """Cascaded initialisation (Eq. 3): per point, the model branch if its voxel's prediction is
    valid, else the PCA branch if the voxel is geometrically reliable (R from the eigenvectors,
    s = s_pca + log beta, Eq. 5), else the heuristic branch (R = I, s = log(d / f), Eq. 6).
    beta: None = per segment, clamp(1 - rho, 0.5, 1) with rho the fraction of the segment's points
    that are reliable but lack a valid prediction; or one fixed value.
    anchored: the model branch keeps only the predicted axis ratio a = exp(s - max s) and anchors it
    at the point's depth, s = log((d / f) a) (Eq. 4).
    Returns Gaussian parameters (component-major [c][N] float64) and the branch per point
    (0 model, 1 PCA, 2 heuristic)."""
    P = np.asarray(points, np.float64)
    N = P.shape[0]
    v = vox["voxel"]
    rel = vox["reliable"][v]
    valid = prediction_valid(pred)[v] if pred is not None else np.zeros(N, bool)
    seg = np.asarray(segment, np.int64)
    if beta is None:
        nseg = int(seg.max()) + 1 if N else 0
        cnt = np.bincount(seg, minlength=nseg).astype(np.float64)
        fb = np.bincount(seg, weights=(rel & ~valid).astype(np.float64), minlength=nseg)
        rho = np.where(cnt > 0, fb / np.maximum(cnt, 1), 0.0)
        b = np.clip(1.0 - rho, 0.5, 1.0)[seg]
    else:
        b = np.full(N, float(beta))
    branch = np.where(valid, 0, np.where(rel, 1, 2))
    ls = np.zeros((3, N))
    qs = np.zeros((4, N))
    lo = np.full(N, np.log(OPACITY_CONST / (1 - OPACITY_CONST)))
    qpca = rot_to_quat(vox["R"])
    for i in range(N):
        if branch[i] == 0:
            p = pred[v[i]]
            ls[:, i] = p[:3]
            if anchored:
                ls[:, i] = np.log(depth[i] / f) + (p[:3] - np.max(p[:3]))
            qs[:, i] = p[3:7] / np.linalg.norm(p[3:7])
            lo[i] = p[7]
        elif branch[i] == 1:
            ls[:, i] = vox["s_pca"][v[i]] + np.log(b[i])
            qs[:, i] = qpca[v[i]]
        else:
            ls[:, i] = np.log(depth[i] / f)
            qs[:, i] = (1.0, 0.0, 0.0, 0.0)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((3 * K, N))
    sh[0:3] = ((np.asarray(colors, np.float64) - 0.5) / Y00).T
    return dict(means=P.T.copy(), log_scales=ls, quats=qs, opacity_logits=lo, sh=sh, sh_degree=sh_degree,
                branch=branch, beta=b)


def descriptor_covariance(points, vox, point_cov):
    """Eq. 1-2 with per-point world covariances.  point_cov [n, 6] = (xx, xy, xz, yy, yz, zz).
    For each planar / linear voxel: J_i = [V F_i; I/N] with V = [v_min v_mid v_max] (the
    canonical frame's columns) and F_i's rows f^(m) = (p_i - mu)^T (v_m v_k^T + v_k v_m^T) /
    (N (lambda_k - lambda_m)) for m != k (zero for m = k), k the descriptor direction (v_min for
    planar, v_max for linear); Sigma_g = sum_i J_i Sigma_i J_i^T over the voxel's fitting points.
    Returns Sigma_g [V, 6, 6] (zero for unreliable-class voxels), the direction-block trace
    (infinity for them) and reliable = class planar / linear and trace < 0.1^2."""
    P = np.asarray(points, np.float64)
    c6 = np.asarray(point_cov, np.float32).astype(np.float64)
    S = np.stack([np.stack([c6[:, 0], c6[:, 1], c6[:, 2]], -1), np.stack([c6[:, 1], c6[:, 3], c6[:, 4]], -1),
                  np.stack([c6[:, 2], c6[:, 4], c6[:, 5]], -1)], -2)
    nv = len(vox["n"])
    Sg = np.zeros((nv, 6, 6))
    tr = np.full(nv, np.inf)
    for v in range(nv):
        if vox["cls"][v] == UNRELIABLE:
            continue
        Vm = vox["R"][v][:, ::-1]               # columns v_min, v_mid, v_max
        lam = vox["evals"][v]
        k = 0 if vox["cls"][v] == PLANAR else 2
        ids = vox["ids"][v]
        N = len(ids)
        for i in ids:
            d = P[i] - vox["mu"][v]
            F = np.zeros((3, 3))
            for m in range(3):
                if m != k:
                    F[m] = d @ (np.outer(Vm[:, m], Vm[:, k]) + np.outer(Vm[:, k], Vm[:, m])) / (N * (lam[k] - lam[m]))
            J = np.concatenate([Vm @ F, np.eye(3) / N])
            Sg[v] += J @ S[i] @ J.T
        tr[v] = np.trace(Sg[v][:3, :3])
    reliable = (vox["cls"] != UNRELIABLE) & (tr < REL_TRACE)
    return Sg, tr, reliable
