"""FP64 oracle of the Gaussian-based loop registration (Sec. III-D, Eq. 13-16).  Test
infrastructure only: the test-suite, the smoke check and the benchmark's CPU baseline may use
it; the product path never imports it.

Definitions (plain, no acceleration structure; every geometric quantity in float64 from the
float32 inputs, each operation rounded separately in the order written, so that the integer
decisions can be compared exactly):

* camera k (world -> camera p = R mu + t): centre c = -R^T t;  projection u = fx (x / z) + cx,
  v = fy (y / z) + cy, inside the image when z > z_near and 0 <= u < W, 0 <= v < H.
* source set: the Gaussians of the loopframe's segment (segment id == src_segment).
* target set (Eq. 13): Gaussians outside the source set for which some query keyframe k both sees
  the mean inside its image and has its centre within d_max of the mean (|mu - c|^2 < d_max^2).
* regularised covariance: the Gaussian's covariance R_q S^2 R_q^T with its eigenvalues replaced by
  (1, 1, 1e-3), the 1e-3 on the axis of the smallest scale (first such axis on ties).
* correspondences: source mean m, moved by the current T = (R, t), pairs with the nearest target
  mean strictly within d_corr (smallest squared distance, lowest target row on ties), or none.
* residual and covariance (Eq. 14, 15): r = mu_n - (R mu_m + t), C = S_n + R S_m R^T, evaluated at
  the current T and not differentiated (the usual GICP linearisation).
* Gauss-Newton on Eq. 16 with the left perturbation T <- (Exp(phi) R, Exp(phi) t + rho),
  xi = (rho, phi): J = dr/dxi = [-I, [q]x] with q = R mu_m + t; H = sum J^T W J, g = sum J^T W r,
  W = C^-1; xi = -H^-1 g.  Converged when a step is below |rho| < 2.5e-3 m and |phi| < 2.5e-4 rad
  (an eighth of the 2 cm range noise): with nearest-neighbour pairing the iterates can end in a
  cycle of two correspondence sets a millimetre apart, so a tighter test would never fire.
* acceptance: converged, at least 100 correspondences, and mean r^T W r below 1.
"""
from __future__ import annotations

import numpy as np

REG_EIG = (1.0, 1.0, 1e-3)
EPS_RHO, EPS_PHI = 2.5e-3, 2.5e-4
MIN_CORR = 100
ACCEPT_COST = 1.0


def _f64(a):
    return np.asarray(a, np.float32).astype(np.float64)


def camera_center(cam):
    R = _f64(np.asarray(cam["R"]).reshape(3, 3))
    t = _f64(cam["t"])
    return np.array([-((R[0, 0] * t[0] + R[1, 0] * t[1]) + R[2, 0] * t[2]),
                     -((R[0, 1] * t[0] + R[1, 1] * t[1]) + R[2, 1] * t[2]),
                     -((R[0, 2] * t[0] + R[1, 2] * t[1]) + R[2, 2] * t[2])])


def _transform(R, t, P):
    """R P + t for P [3, n], each coordinate ((R0 x + R1 y) + R2 z) + t."""
    return np.stack([((R[i, 0] * P[0] + R[i, 1] * P[1]) + R[i, 2] * P[2]) + t[i] for i in range(3)])


def _sqdist(A, b):
    """Squared distances ((dx^2 + dy^2) + dz^2) between the columns of A and the point b."""
    dx, dy, dz = A[0] - b[0], A[1] - b[1], A[2] - b[2]
    return (dx * dx + dy * dy) + dz * dz


def source_set(segment_id, src_segment):
    return np.asarray(segment_id) == src_segment


def target_set(means, segment_id, src_segment, cams, d_max):
    """Eq. 13: bool [n]."""
    M = _f64(means)
    keep = np.zeros(M.shape[1], bool)
    dd = np.float64(np.float32(d_max)) ** 2
    for cam in cams:
        R = _f64(np.asarray(cam["R"]).reshape(3, 3))
        t = _f64(cam["t"])
        p = _transform(R, t, M)
        x, y, z = p
        front = z > np.float64(np.float32(cam["z_near"]))
        with np.errstate(divide="ignore", invalid="ignore"):
            u = np.float64(np.float32(cam["fx"])) * (x / z) + np.float64(np.float32(cam["cx"]))
            v = np.float64(np.float32(cam["fy"])) * (y / z) + np.float64(np.float32(cam["cy"]))
        inside = front & (u >= 0) & (u < cam["width"]) & (v >= 0) & (v < cam["height"])
        near = _sqdist(M, camera_center(cam)) < dd
        keep |= inside & near
    return keep & ~source_set(segment_id, src_segment)


def quat_to_rot(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                     np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                     np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def regularized_cov(quats, log_scales):
    """[n, 3, 3]: R_q diag(l) R_q^T with l = 1e-3 on the smallest-scale axis, 1 elsewhere."""
    R = quat_to_rot(_f64(quats).T)                      # [n, 3, 3], columns = axes
    s = _f64(log_scales).T                               # [n, 3]
    a = np.argmin(s, axis=1)
    lam = np.ones_like(s)
    lam[np.arange(s.shape[0]), a] = REG_EIG[2]
    return np.einsum("nij,nj,nkj->nik", R, lam, R)


def correspondences(q, tgt, d_corr):
    """q [3, m] moved source means, tgt [3, k] target means: index into tgt or -1."""
    dd = np.float64(np.float32(d_corr)) ** 2
    out = np.full(q.shape[1], -1, np.int64)
    if tgt.shape[1] == 0:
        return out
    for j in range(q.shape[1]):
        d2 = _sqdist(tgt, q[:, j])
        i = int(np.argmin(d2))  # first minimum: lowest target row on ties
        if d2[i] < dd:
            out[j] = i
    return out


def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def normal_equations(R, t, src_means, src_cov, tgt_means, tgt_cov, d_corr):
    """One linearisation of Eq. 16 at T = (R, t).  Returns dict H [6, 6], g [6], cost, sq
    (sum |r|^2), count, corr."""
    S = _f64(src_means)
    T = _f64(tgt_means)
    q = _transform(R, t, S)
    corr = correspondences(q, T, d_corr)
    H = np.zeros((6, 6))
    g = np.zeros(6)
    cost = sq = 0.0
    count = 0
    for m in np.nonzero(corr >= 0)[0]:
        n = corr[m]
        r = T[:, n] - q[:, m]
        C = tgt_cov[n] + R @ src_cov[m] @ R.T
        W = np.linalg.inv(C)
        J = np.concatenate([-np.eye(3), skew(q[:, m])], axis=1)
        H += J.T @ W @ J
        g += J.T @ W @ r
        cost += r @ W @ r
        sq += r @ r
        count += 1
    return dict(H=H, g=g, cost=cost, sq=sq, count=count, corr=corr)


def so3_exp(phi):
    th = np.linalg.norm(phi)
    K = skew(phi)
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1 - np.cos(th)) / th ** 2 * K @ K


def gn_update(R, t, H, g):
    xi = -np.linalg.solve(H, g)
    E = so3_exp(xi[3:])
    return E @ R, E @ t + xi[:3], xi


def register(R0, t0, src_means, src_cov, tgt_means, tgt_cov, d_corr, max_iter=30):
    """Gauss-Newton from (R0, t0).  Returns dict R, t, converged, iterations, the last linearisation's
    statistics, accepted."""
    R, t = np.asarray(R0, np.float64), np.asarray(t0, np.float64)
    conv = False
    it = 0
    ne = None
    for it in range(1, max_iter + 1):
        ne = normal_equations(R, t, src_means, src_cov, tgt_means, tgt_cov, d_corr)
        if ne["count"] < 6:
            break
        R, t, xi = gn_update(R, t, ne["H"], ne["g"])
        if np.linalg.norm(xi[:3]) < EPS_RHO and np.linalg.norm(xi[3:]) < EPS_PHI:
            conv = True
            break
    accepted = bool(conv and ne["count"] >= MIN_CORR and ne["cost"] / ne["count"] < ACCEPT_COST)
    return dict(R=R, t=t, converged=conv, iterations=it, stats=ne, accepted=accepted)


# ---- propagation of a corrected pose to a segment (Sec. III-D, last paragraph) ---------------------
#
# The segment's Gaussians move rigidly with the world-frame transform (R, t): means R mu + t,
# orientations R R_q (quaternion q_R (x) q), and the view-dependent colour rotates with them:
# colour'(R d) = colour(d), i.e. the new SH coefficients of each degree are the least-squares fit
# of the old colour function sampled at R^T d.  The segment's cameras (world -> camera R_c, t_c)
# move with it: R_c R^T, t_c - R_c R^T t.

def rot_to_quat(R):
    """Unit quaternion (w, x, y, z) of a rotation matrix (scipy's conversion), sign chosen w >= 0."""
    from scipy.spatial.transform import Rotation
    x, y, z, w = Rotation.from_matrix(np.asarray(R, np.float64)).as_quat()
    q = np.array([w, x, y, z])
    return -q if w < 0 else q


def quat_mul(a, b):
    """Hamilton product a (x) b for (w, x, y, z) quaternions; b may be [4, n]."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def sh_rotation_fit(R, degree, n_dirs=400, seed=0):
    """Per degree l >= 1, the matrix D_l with c' = D_l c such that sum_a c'_a Y_a(d) =
    sum_b c_b Y_b(R^T d) for every direction d: the least-squares solution of Y D = Y_rot over
    random directions (exact, since each degree's span is closed under rotation)."""
    import oracle
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n_dirs, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y, _ = oracle.sh_basis(degree, d)                 # [n_dirs, K]
    Yr, _ = oracle.sh_basis(degree, d @ np.asarray(R))  # rows R^T d
    out = {}
    for l in range(1, degree + 1):
        s = slice(l * l, (l + 1) * (l + 1))
        # Y[:, s] D = Yr[:, s]  =>  new coefficients c' = D c
        D, *_ = np.linalg.lstsq(Y[:, s], Yr[:, s], rcond=None)
        out[l] = D
    return out


def transform_segment(g, segment_id, segment, R, t):
    """New means [3, n], quats [4, n] and sh [3K, n] (float64) with the segment moved by (R, t)."""
    R, t = np.asarray(R, np.float64), np.asarray(t, np.float64)
    sel = np.asarray(segment_id) == segment
    means = _f64(g["means"]).copy()
    quats = _f64(g["quats"]).copy()
    sh = _f64(g["sh"]).copy()
    means[:, sel] = R @ means[:, sel] + t[:, None]
    quats[:, sel] = quat_mul(rot_to_quat(R), quats[:, sel])
    deg = int(g["sh_degree"])
    D = sh_rotation_fit(R, deg) if deg > 0 else {}
    K = (deg + 1) ** 2
    old = sh.reshape(K, 3, -1)
    new = old.copy()
    for l, Dl in D.items():
        s = slice(l * l, (l + 1) * (l + 1))
        blk = new[s]
        blk[:, :, sel] = np.einsum("ab,bcn->acn", Dl, old[s][:, :, sel])
        new[s] = blk
    return means, quats, new.reshape(3 * K, -1)


def transform_camera(cam, R, t):
    Rc = _f64(np.asarray(cam["R"]).reshape(3, 3))
    tc = _f64(cam["t"])
    R, t = np.asarray(R, np.float64), np.asarray(t, np.float64)
    return Rc @ R.T, tc - Rc @ R.T @ t
