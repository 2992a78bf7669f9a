"""Pins of the oracle's learned-initialisation helpers (Sec. III-B, Eq. 3) against hand-built
cases: the network's per-voxel inputs (cyclic rows, centring and scale, the 12 features in their
stated order), the per-voxel training targets (brute-force loop over the Gaussians of each voxel,
rotations from scipy), and the bounds of Eq. 3's "valid prediction" one float32 step inside and
outside log 2 mm and log 0.5 m."""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import init_oracle as io
from oracle import pointnet_oracle as pn


def _hand_voxels():
    """Two voxels built by hand (not by voxel_pca): voxel 0 holds 3 fitting points, voxel 1 holds
    32; R's columns are (v_max, v_mid, v_min)."""
    P = np.zeros((40, 3))
    P[[4, 9, 2]] = [[1.0, 2.0, 3.0], [1.5, 2.0, 3.0], [1.0, 2.25, 3.5]]
    rng = np.random.default_rng(3)
    ids1 = np.arange(10, 40)[::-1][:30].tolist() + [0, 1]          # 32 ids in a deliberate order
    P[ids1] = rng.uniform(-2, 2, (32, 3))
    mu0 = np.array([1.0, 2.0, 3.0])
    mu1 = P[ids1].mean(axis=0)
    R0 = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])   # v_max=e_y, v_mid=e_z, v_min=e_x
    c, s = np.cos(0.3), np.sin(0.3)
    R1 = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    vox = dict(n=np.array([3, 32]), ids=[np.array([4, 9, 2]), np.array(ids1)], mu=np.stack([mu0, mu1]),
               evals=np.array([[1e-6, 0.01, 0.25], [0.0025, 0.04, 1.0]]), R=np.stack([R0, R1]))
    return P, vox


def test_voxel_inputs_rows_repeat_cyclically_and_are_centred_and_scaled():
    P, vox = _hand_voxels()
    X, F = pn.voxel_inputs(P, vox)
    assert X.shape == (2, 32, 3) and F.shape == (2, 12)
    # voxel 0: rows 0, 1, 2, 3, ... are points 4, 9, 2, 4, 9, 2, ... minus the mean, over 0.5 m
    expect = {0: [0.0, 0.0, 0.0], 1: [1.0, 0.0, 0.0], 2: [0.0, 0.5, 1.0]}
    for r in range(32):
        np.testing.assert_array_equal(X[0, r], expect[r % 3])
    # voxel 1: 32 points, each row once in the listed order
    ids1 = vox["ids"][1]
    for r in range(32):
        np.testing.assert_allclose(X[1, r], (P[ids1[r]] - vox["mu"][1]) * 2.0, rtol=0, atol=1e-15)


def test_voxel_features_order_and_scale():
    P, vox = _hand_voxels()
    _, F = pn.voxel_inputs(P, vox)
    # eigenvalues ascending, floored at (5 mm)^2, as log(lambda / (0.5 m)^2)
    np.testing.assert_allclose(F[0, 0:3], [np.log(2.5e-5 / 0.25), np.log(0.04), 0.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(F[1, 0:3], [np.log(0.01), np.log(0.16), np.log(4.0)], rtol=0, atol=1e-15)
    # then v_min, v_mid, v_max: R's columns in reverse order
    np.testing.assert_array_equal(F[0, 3:6], [1.0, 0.0, 0.0])     # e_x
    np.testing.assert_array_equal(F[0, 6:9], [0.0, 0.0, 1.0])     # e_z
    np.testing.assert_array_equal(F[0, 9:12], [0.0, 1.0, 0.0])    # e_y
    c, s = np.cos(0.3), np.sin(0.3)
    np.testing.assert_array_equal(F[1, 3:6], [0.0, 0.0, 1.0])
    np.testing.assert_allclose(F[1, 6:9], [-s, c, 0.0])
    np.testing.assert_allclose(F[1, 9:12], [c, s, 0.0])


def test_voxel_inputs_follow_the_fitted_selection():
    """On a voxel_pca fit: each voxel's rows are its selected points (ascending hash) in order."""
    rng = np.random.default_rng(8)
    pts = np.concatenate([rng.uniform(0.01, 0.49, (50, 3)), rng.uniform([1.01, 0.01, 0.01], [1.49, 0.49, 0.49],
                                                                         (7, 3))])
    vox = io.voxel_pca(pts, seed=5)
    X, _ = pn.voxel_inputs(pts, vox)
    for v in range(len(vox["n"])):
        ids = vox["ids"][v]
        assert len(ids) == min(32, vox["n_all"][v])
        for r in range(32):
            np.testing.assert_allclose(X[v, r] * 0.5 + vox["mu"][v], pts[ids[r % len(ids)]], atol=1e-12)


def _cov_bruteforce(s, q_wxyz):
    R = Rotation.from_quat([q_wxyz[1], q_wxyz[2], q_wxyz[3], q_wxyz[0]]).as_matrix()  # normalises
    return R @ np.diag(np.exp(2.0 * np.asarray(s))) @ R.T


def test_targets_from_gaussians_brute_force():
    # 3 voxels: voxel 0 receives Gaussians 0 and 2, voxel 1 none, voxel 2 Gaussian 1 (and 3, which
    # was seeded from a point of voxel 2 as well)
    vox = dict(n=np.array([2, 1, 3]), voxel=np.array([0, 2, 0, 1, 2, 2]))
    point_ids = np.array([0, 4, 2, 5])
    ls = np.array([[-2.0, -1.0, -3.0], [-1.5, -1.5, -1.5], [-3.0, -2.5, -2.0], [-1.0, -4.0, -2.0]]).T
    q = np.array([[2.0, 0.0, 0.0, 0.0], [0.9, 0.1, -0.3, 0.2], [0.1, 0.7, 0.2, -0.4], [0.5, 0.5, 0.5, 0.5]]).T
    lo = np.array([0.3, -1.2, 2.0, 0.0])
    ct, ot, has = pn.targets_from_gaussians(vox, ls, q, lo, point_ids)
    assert has.tolist() == [True, False, True]
    members = {0: [0, 2], 2: [1, 3]}
    for v, gs in members.items():
        cov = sum(_cov_bruteforce(ls[:, g], q[:, g]) for g in gs) / len(gs)
        op = sum(1.0 / (1.0 + np.exp(-lo[g])) for g in gs) / len(gs)
        np.testing.assert_allclose(ct[v], cov, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(ot[v], op, rtol=1e-12)
    np.testing.assert_array_equal(ct[1], np.zeros((3, 3)))
    assert ot[1] == 0.0
    # closed form: an unrotated Gaussian (q not normalised) with scale 0.1 m has covariance 0.01 I
    np.testing.assert_allclose(_cov_bruteforce([np.log(0.1)] * 3, [2, 0, 0, 0]), 0.01 * np.eye(3), atol=1e-15)
    ct1, ot1, _ = pn.targets_from_gaussians(dict(n=np.array([1]), voxel=np.array([0])),
                                            np.full((3, 1), np.log(0.1)), np.array([[3.0], [0], [0], [0]]),
                                            np.array([0.0]), np.array([0]))
    np.testing.assert_allclose(ct1[0], 0.01 * np.eye(3), rtol=1e-13)
    assert ot1[0] == 0.5


def _pred(s):
    p = np.zeros((len(s), 8))
    p[:, :3] = np.asarray(s)[:, None]
    p[:, 3] = 1.0
    return p


def test_prediction_valid_bounds():
    # the decision is taken in float32, the precision of the network's outputs
    lo32 = np.float32(np.log(0.002))
    hi32 = np.float32(np.log(0.5))
    below = np.nextafter(lo32, np.float32(-np.inf))
    above = np.nextafter(hi32, np.float32(np.inf))
    s = np.array([lo32, below, hi32, above, np.nextafter(lo32, np.float32(0)), np.nextafter(hi32, np.float32(-1))],
                 np.float32).astype(np.float64)
    assert io.prediction_valid(_pred(s)).tolist() == [True, False, True, False, True, True]
    # plain cases on both sides of each bound: 2 mm and 0.5 m, not 2 cm or 5 m
    s2 = np.log([0.0019, 0.0021, 0.005, 0.019, 0.3, 0.49, 0.51, 2.0])
    assert io.prediction_valid(_pred(s2)).tolist() == [False, True, True, True, True, True, False, False]
    # one axis out of range is enough; a zero quaternion and non-finite outputs are invalid
    p = _pred([np.log(0.01)] * 5)
    p[0, 1] = np.log(0.6)
    p[1, 3:7] = 0.0
    p[2, 7] = np.nan
    p[3, 4] = np.inf
    assert io.prediction_valid(p).tolist() == [False, False, False, False, True]
