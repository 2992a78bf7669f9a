"""Pins of the loop-registration oracle (Sec. III-D, Eq. 13-16): the regularised covariance
against an eigendecomposition, the target set on hand-placed points, nearest correspondences
against scipy's k-d tree, the normal equations against finite-difference Jacobians, and exact
recovery of a known rigid transform."""
import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import synth
from oracle import gicp_oracle as go


def _gaussians(rng, n):
    q = rng.standard_normal((4, n)).astype(np.float32)
    s = rng.normal(-3, 0.7, (3, n)).astype(np.float32)
    return q, s


def test_regularized_cov_replaces_the_eigenvalues():
    rng = np.random.default_rng(0)
    q, s = _gaussians(rng, 200)
    S = go.regularized_cov(q, s)
    R = go.quat_to_rot(q.astype(np.float64).T)
    cov = np.einsum("nij,nj,nkj->nik", R, np.exp(2 * s.astype(np.float64).T), R)
    lam, V = np.linalg.eigh(cov)              # ascending: column 0 is the smallest-scale axis
    exp = np.einsum("nij,nj,nkj->nik", V, np.tile([1e-3, 1.0, 1.0], (200, 1)), V)
    np.testing.assert_allclose(S, exp, atol=1e-12)
    # closed form: I - (1 - 1e-3) a a^T with a the smallest-scale axis
    a = R[np.arange(200), :, np.argmin(s, axis=0)]
    np.testing.assert_allclose(S, np.eye(3) - 0.999 * np.einsum("ni,nj->nij", a, a), atol=1e-12)


def test_target_set_hand_cases():
    cam = synth.make_camera(np.eye(3), np.zeros(3), 100.0, 100.0, 50.0, 40.0, 100, 80)
    means = np.array([[0.0, 0.0, 5.0],     # centre of view, 5 m
                      [0.0, 0.0, 25.0],    # in view, beyond d_max
                      [3.0, 0.0, 5.0],     # outside the image (u = 110)
                      [0.0, 0.0, -5.0],    # behind
                      [0.0, 0.0, 6.0],     # in view but in the source segment
                      [-2.5, -2.0, 5.0],   # u = 0, v = 0: the image's first pixel corner, inside
                      [2.5, 0.0, 5.0]],    # u = 100 = W: outside
                     np.float32).T
    seg = np.array([0, 0, 0, 0, 7, 0, 0])
    got = go.target_set(means, seg, 7, [cam], 20.0)
    assert got.tolist() == [True, False, False, False, False, True, False]
    cam2 = synth.make_camera(np.eye(3), np.array([0.0, 0.0, -20.0]), 100.0, 100.0, 50.0, 40.0, 100, 80)
    got = go.target_set(means, seg, 7, [cam, cam2], 20.0)  # the second camera sits at z = 20
    assert got.tolist() == [True, True, False, False, False, True, False]


def test_correspondences_match_kdtree():
    rng = np.random.default_rng(1)
    T = rng.uniform(-3, 3, (3, 3000))
    Q = rng.uniform(-3, 3, (3, 400))
    d = 0.3
    c = go.correspondences(Q, T, d)
    dist, idx = cKDTree(T.T).query(Q.T)
    ok = np.abs(dist - d) > 1e-9
    assert np.array_equal((c >= 0)[ok], (dist < d)[ok])
    hit = (c >= 0) & ok
    assert np.array_equal(c[hit], idx[hit])
    assert 50 < hit.sum() < 400


def _surface_scene(rng, n):
    """Means on three orthogonal planes and a box, with flat Gaussians aligned to the surfaces."""
    pts, nrm = [], []
    for k in range(n):
        f = rng.integers(4)
        a, b = rng.uniform(-4, 4, 2)
        if f == 0:
            p, nv = [a, b, -1.0], [0, 0, 1]
        elif f == 1:
            p, nv = [a, 3.0, b], [0, 1, 0]
        elif f == 2:
            p, nv = [-3.0, a, b], [1, 0, 0]
        else:
            p, nv = [1 + 0.5 * np.cos(a), 0.5 * np.sin(a), b * 0.2], [np.cos(a), np.sin(a), 0]
        pts.append(p)
        nrm.append(nv)
    P = np.array(pts, np.float64).T
    Nn = np.array(nrm, np.float64)
    # quaternion whose third axis (smallest scale) is the normal
    rots = []
    for nv in Nn:
        z = nv / np.linalg.norm(nv)
        x = np.cross(z, [0.3, 0.5, 0.8])
        x /= np.linalg.norm(x)
        rots.append(np.stack([x, np.cross(z, x), z], 1))
    q = Rotation.from_matrix(np.array(rots)).as_quat()  # x, y, z, w
    quat = np.stack([q[:, 3], q[:, 0], q[:, 1], q[:, 2]]).astype(np.float32)
    s = np.tile(np.array([[-2.5], [-2.5], [-5.0]]), (1, n)).astype(np.float32)
    return P.astype(np.float32), quat, s


def test_normal_equations_match_finite_difference_jacobians():
    rng = np.random.default_rng(2)
    P, q, s = _surface_scene(rng, 600)
    cov = go.regularized_cov(q, s)
    R0 = Rotation.from_rotvec([0.02, -0.01, 0.03]).as_matrix()
    t0 = np.array([0.05, -0.03, 0.02])
    src = P[:, :300]
    ne = go.normal_equations(R0, t0, src, cov[:300], P[:, 300:], cov[300:], 0.8)
    assert ne["count"] > 100
    S, T = src.astype(np.float32).astype(np.float64), P[:, 300:].astype(np.float32).astype(np.float64)
    H, g = np.zeros((6, 6)), np.zeros(6)
    h = 1e-6
    for m in np.nonzero(ne["corr"] >= 0)[0]:
        n = ne["corr"][m]

        def res(xi):
            E = go.so3_exp(xi[3:])
            return T[:, n] - (E @ (R0 @ S[:, m] + t0) + xi[:3])
        J = np.stack([(res(h * e) - res(-h * e)) / (2 * h) for e in np.eye(6)], 1)
        W = np.linalg.inv(cov[300 + n] + R0 @ cov[m] @ R0.T)
        H += J.T @ W @ J
        g += J.T @ W @ res(np.zeros(6))
    np.testing.assert_allclose(ne["H"], H, rtol=1e-6, atol=1e-6 * np.abs(H).max())
    np.testing.assert_allclose(ne["g"], g, rtol=1e-6, atol=1e-6 * np.abs(g).max())


def test_register_recovers_a_known_transform():
    rng = np.random.default_rng(3)
    P, q, s = _surface_scene(rng, 1500)
    cov = go.regularized_cov(q, s)
    Rt = Rotation.from_rotvec([0.03, -0.02, 0.05]).as_matrix()
    tt = np.array([0.12, -0.08, 0.05])
    # source: a subset of the same Gaussians, moved by the inverse of (Rt, tt)
    idx = rng.choice(1500, 600, replace=False)
    Pd = P.astype(np.float64)
    src = Rt.T @ (Pd[:, idx] - tt[:, None])
    src_cov = np.einsum("ij,njk,lk->nil", Rt.T, cov[idx], Rt.T)
    src32 = src.astype(np.float32)
    out = go.register(np.eye(3), np.zeros(3), src32, src_cov, P, cov, 0.5)
    assert out["converged"] and out["accepted"]
    # the float32 rounding of the moved source means bounds the recovery
    assert np.abs(out["R"] - Rt).max() < 1e-5 and np.abs(out["t"] - tt).max() < 1e-5
    assert out["stats"]["cost"] / out["stats"]["count"] < 1e-6


def test_segment_transform_moves_geometry_and_colour():
    import oracle
    rng = np.random.default_rng(4)
    g = synth.random_gaussians(5, 300, 3)
    seg = rng.integers(0, 3, 300)
    R = Rotation.from_rotvec([0.3, -0.2, 0.5]).as_matrix()
    t = np.array([1.0, -2.0, 0.5])
    means, quats, sh = go.transform_segment(g, seg, 1, R, t)
    sel = seg == 1
    m0 = g["means"].astype(np.float64)
    np.testing.assert_allclose(means[:, sel], R @ m0[:, sel] + t[:, None], atol=1e-12)
    np.testing.assert_array_equal(means[:, ~sel], m0[:, ~sel])
    # orientation: R_q' = R R_q, magnitude of the raw quaternion kept
    Rq0 = go.quat_to_rot(g["quats"].astype(np.float64).T)
    Rq1 = go.quat_to_rot(quats.T)
    np.testing.assert_allclose(Rq1[sel], np.einsum("ij,njk->nik", R, Rq0[sel]), atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(quats, axis=0), np.linalg.norm(g["quats"].astype(np.float64), axis=0),
                               rtol=1e-12)
    # colour seen along R d after the move equals the colour seen along d before it
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y0, _ = oracle.sh_basis(3, d)
    Y1, _ = oracle.sh_basis(3, d @ R.T)
    old = g["sh"].astype(np.float64).reshape(16, 3, -1)
    new = sh.reshape(16, 3, -1)
    for i in np.nonzero(sel)[0][:20]:
        np.testing.assert_allclose(Y1 @ new[:, :, i], Y0 @ old[:, :, i], atol=1e-10)
    # each degree's matrix is orthogonal and the map is a representation: D(R1 R2) = D(R1) D(R2)
    R2 = Rotation.from_rotvec([-0.1, 0.4, 0.2]).as_matrix()
    D1, D2, D12 = go.sh_rotation_fit(R, 3), go.sh_rotation_fit(R2, 3), go.sh_rotation_fit(R @ R2, 3)
    for l in (1, 2, 3):
        np.testing.assert_allclose(D1[l] @ D1[l].T, np.eye(2 * l + 1), atol=1e-10)
        np.testing.assert_allclose(D12[l], D1[l] @ D2[l], atol=1e-10)
    # the segment's camera moves with it: a moved point projects where the old one did
    cam = synth.make_camera(Rotation.from_rotvec([0.1, 0.2, -0.3]).as_matrix(), [0.3, 0.1, 2.0], 100, 100, 50, 40,
                            100, 80)
    Rc, tc = go.transform_camera(cam, R, t)
    p = rng.standard_normal(3)
    np.testing.assert_allclose(Rc @ (R @ p + t) + tc, cam["R"].astype(np.float64) @ p + cam["t"].astype(np.float64),
                               atol=1e-6)
