"""Pins of the initialisation oracle (voxel PCA, Sec. III-A; cascade, Sec. III-B) against
published test vectors, library routines, closed forms and brute force."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import init_oracle as io
import synth


def test_splitmix64_published_sequence():
    # the first outputs of SplitMix64 started from state 0 (the reference generator's sequence)
    g = 0x9E3779B97F4A7C15
    got = io.splitmix64(np.array([0, g, (2 * g) % 2 ** 64], dtype=np.uint64))
    assert [int(x) for x in got] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_jacobi_matches_numpy_eigh():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((200, 3, 3))
    C = A @ np.transpose(A, (0, 2, 1)) + 1e-3 * np.eye(3)
    C[:20] = np.diag([1.0, 1.0, 2.0])  # repeated eigenvalues
    lam, V = io.jacobi_eigh3(C)
    lam_ref, V_ref = np.linalg.eigh(C)
    np.testing.assert_allclose(lam, lam_ref, rtol=1e-12, atol=1e-13)
    # reconstruction and orthonormality (eigenvectors of repeated eigenvalues are not unique)
    np.testing.assert_allclose(V @ (lam[:, :, None] * np.transpose(V, (0, 2, 1))), C, atol=1e-12)
    np.testing.assert_allclose(np.transpose(V, (0, 2, 1)) @ V, np.broadcast_to(np.eye(3), V.shape), atol=1e-12)
    simple = np.min(np.diff(lam_ref, axis=1), axis=1) > 1e-6
    dots = np.abs(np.einsum("nij,nij->nj", V, V_ref))
    np.testing.assert_allclose(dots[simple], 1.0, atol=1e-10)


def test_planar_patch_closed_form():
    # points on the plane with normal n, noise sigma along n: lambda_min -> sigma^2, v_min -> n
    rng = np.random.default_rng(1)
    n = np.array([0.3, -0.2, 0.93])
    n /= np.linalg.norm(n)
    u = np.cross(n, [1.0, 0, 0])
    u /= np.linalg.norm(u)
    w = np.cross(n, u)
    sigma = 0.01
    m = 20000
    pts = (np.array([0.25, 0.25, 0.25]) + rng.uniform(-0.2, 0.2, (m, 1)) * u + rng.uniform(-0.2, 0.2, (m, 1)) * w
           + rng.normal(0, sigma, (m, 1)) * n)
    C = np.cov(pts.T, bias=True)
    lam, V = io.jacobi_eigh3(C[None])
    assert abs(lam[0, 0] / sigma ** 2 - 1) < 0.05
    assert abs(abs(V[0, :, 0] @ n) - 1) < 1e-4
    vox = io.voxel_pca(pts[:400], seed=3)
    assert len(vox["cls"]) == 1 and vox["cls"][0] == io.PLANAR and vox["n"][0] == 32 and vox["reliable"][0]


def test_thick_segment_is_linear():
    rng = np.random.default_rng(2)
    t = rng.uniform(-0.22, 0.22, 2000)
    pts = np.array([0.25, 0.25, 0.25]) + t[:, None] * np.array([1.0, 0, 0]) + rng.normal(0, 0.06, (2000, 3)) * [0, 1, 1]
    pts = pts[np.all((pts >= 0) & (pts < 0.5), axis=1)]
    vox = io.voxel_pca(pts, seed=1)
    assert len(vox["cls"]) == 1
    lam = vox["evals"][0]
    assert lam[0] >= io.TAU_P and lam[2] / lam[0] > io.TAU_L
    assert vox["cls"][0] == io.LINEAR
    assert abs(abs(vox["R"][0][:, 0] @ [1.0, 0, 0]) - 1) < 0.05  # v_max along the segment


def test_direction_trace_closed_form():
    # Eq. 1-2 summed over points equals sigma^2 / N sum_{m != k} (l_m + l_k) / (l_k - l_m)^2,
    # which follows from sum_i (d_i . v_m)^2 = N l_m and d_i . v_m orthogonal components
    rng = np.random.default_rng(3)
    for k in (0, 2):
        d = rng.standard_normal((25, 3)) * [0.3, 0.1, 0.02]
        C = d.T @ d / 25
        lam, V = np.linalg.eigh(C)
        dd = (d - d.mean(0)) @ V
        lam = np.diag(dd.T @ dd / 25)
        tr = io.direction_trace_points(dd, lam, k)
        ref = io.SIGMA_PT ** 2 / 25 * sum((lam[m] + lam[k]) / (lam[k] - lam[m]) ** 2 for m in range(3) if m != k)
        np.testing.assert_allclose(tr, ref, rtol=1e-10)


def test_selection_keeps_smallest_hashes_and_frame_is_canonical():
    rng = np.random.default_rng(4)
    pts = rng.uniform(0, 1.5, (3000, 3))
    seed = 77
    vox = io.voxel_pca(pts, seed)
    key = np.floor(pts / 0.5).astype(int)
    M = (1 << 64) - 1
    for v in range(len(vox["n"])):
        members = [i for i in range(len(pts)) if tuple(key[i]) == tuple(vox["key"][v])]
        # brute force with Python integers: the published SplitMix64 steps, mod 2^64
        def sm(x):
            z = (x + 0x9E3779B97F4A7C15) & M
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
            return z ^ (z >> 31)
        exp = sorted(members, key=lambda i: (sm(seed ^ i), i))[:32]
        assert list(vox["ids"][v]) == exp
        assert vox["n_all"][v] == len(members)
        assert np.all(vox["voxel"][members] == v)
    R = vox["R"]
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)
    np.testing.assert_allclose(np.transpose(R, (0, 2, 1)) @ R, np.broadcast_to(np.eye(3), R.shape), atol=1e-12)
    for j in (0, 1):
        col = R[:, :, j]
        assert np.all(np.take_along_axis(col, np.argmax(np.abs(col), 1)[:, None], 1) > 0)
    # voxels ascend lexicographically
    k = vox["key"]
    assert all(tuple(k[i]) < tuple(k[i + 1]) for i in range(len(k) - 1))


def test_rot_to_quat_matches_scipy():
    R = Rotation.random(300, random_state=5).as_matrix()
    q = io.rot_to_quat(R)
    ref = Rotation.from_matrix(R).as_quat()  # (x, y, z, w)
    ref = np.concatenate([ref[:, 3:], ref[:, :3]], axis=1)
    ref *= np.where(ref[:, :1] < 0, -1.0, 1.0)
    np.testing.assert_allclose(q, ref, atol=1e-12)


def test_cascade_branches():
    # three voxels: planar (reliable), sparse (unreliable), and one with a valid prediction
    rng = np.random.default_rng(6)
    a = np.column_stack([rng.uniform(0.05, 0.45, 40), rng.uniform(0.05, 0.45, 40), 0.25 + rng.normal(0, 0.005, 40)])
    b = np.array([[1.2, 0.2, 0.2], [1.3, 0.3, 0.3], [1.1, 0.4, 0.1]])
    c = np.column_stack([rng.uniform(2.05, 2.45, 40), rng.uniform(0.05, 0.45, 40), 0.25 + rng.normal(0, 0.005, 40)])
    pts = np.concatenate([a, b, c])
    col = rng.uniform(0, 1, (len(pts), 3))
    vox = io.voxel_pca(pts, seed=0)
    assert list(vox["reliable"]) == [True, False, True]
    pred = np.array([[np.nan] * 8, [np.log(0.1)] * 3 + [1, 0, 0, 0, 0.3], [np.log(0.05)] * 3 + [0, 2, 0, 0, 1.5]])
    depth = np.full(len(pts), 6.4)
    seg = np.zeros(len(pts), int)
    g = io.cascade(pts, col, depth, seg, vox, pred=pred, f=640.0)
    br = g["branch"]
    assert np.all(br[:40] == 1) and np.all(br[40:43] == 0) and np.all(br[43:] == 0)
    # the unreliable voxel has a valid prediction: model branch, normalised quaternion
    np.testing.assert_allclose(g["quats"][:, 40], [1, 0, 0, 0])
    np.testing.assert_allclose(g["quats"][:, 43], [0, 1, 0, 0])
    np.testing.assert_allclose(g["opacity_logits"][43], 1.5)
    # PCA branch: beta from the segment's reliable-without-prediction fraction (40 of 83)
    beta = np.clip(1 - 40 / 83, 0.5, 1.0)
    np.testing.assert_allclose(g["log_scales"][:, 0], vox["s_pca"][0] + np.log(beta))
    np.testing.assert_allclose(g["opacity_logits"][0], np.log(0.1 / 0.9))
    # heuristic branch without any model
    g2 = io.cascade(pts, col, depth, seg, vox, pred=None, f=640.0)
    assert np.all(g2["branch"][40:43] == 2)
    np.testing.assert_allclose(g2["log_scales"][:, 41], np.log(6.4 / 640.0))
    np.testing.assert_allclose(g2["quats"][:, 41], [1, 0, 0, 0])
    np.testing.assert_allclose(g2["sh"][0:3, 5], (col[5] - 0.5) / io.Y00)


def _cloud(seed):
    """Two planar patches and a thin bar inside a few voxels, with anisotropic LiDAR covariances."""
    rng = np.random.default_rng(seed)
    a = np.c_[rng.uniform(0.02, 0.48, (300, 2)), 0.25 + rng.normal(0, 0.01, 300)]
    b = np.c_[0.75 + rng.normal(0, 0.01, 300), rng.uniform(0.52, 0.98, (300, 2))]
    c = np.c_[rng.uniform(0.52, 0.98, 200), 0.25 + rng.normal(0, 0.05, 200), 0.25 + rng.normal(0, 0.05, 200)]
    pts = np.concatenate([a, b, c])
    org = np.tile([[3.0, -2.0, 1.8]], (pts.shape[0], 1))
    return pts, synth.lidar_point_cov(pts, org)


def test_descriptor_covariance_isotropic_reduces_to_the_trace():
    pts, _ = _cloud(5)
    vox = io.voxel_pca(pts, 3)
    iso = np.tile(np.array([io.SIGMA_PT ** 2, 0, 0, io.SIGMA_PT ** 2, 0, io.SIGMA_PT ** 2], np.float32), (len(pts), 1))
    Sg, tr, rel = io.descriptor_covariance(pts, vox, iso)
    ok = vox["cls"] != io.UNRELIABLE
    assert ok.sum() >= 2
    # point covariances are float32 inputs: sigma^2 = 4e-4 carries a 2.5e-8 relative rounding
    np.testing.assert_allclose(tr[ok], vox["trace"][ok], rtol=1e-7)
    assert np.array_equal(rel, vox["reliable"])
    for v in np.nonzero(ok)[0]:
        N = vox["n"][v]
        np.testing.assert_allclose(Sg[v][3:, 3:], io.SIGMA_PT ** 2 / N * np.eye(3), rtol=1e-6, atol=1e-15)
        np.testing.assert_allclose(Sg[v], Sg[v].T, atol=1e-18)
        assert np.linalg.eigvalsh(Sg[v]).min() > -1e-15


def test_descriptor_jacobian_matches_finite_differences():
    """J_i of Eq. 1 against central differences of (v_k, mu) through numpy's eigh, per point."""
    import synth as _s  # noqa: F401
    pts, cov = _cloud(6)
    vox = io.voxel_pca(pts, 4)
    Sg, tr, _ = io.descriptor_covariance(pts, vox, cov)
    c6 = cov.astype(np.float64)
    for v in np.nonzero(vox["cls"] != io.UNRELIABLE)[0][:3]:
        ids = vox["ids"][v]
        k = 0 if vox["cls"][v] == io.PLANAR else 2
        vref = vox["R"][v][:, ::-1][:, k]

        def desc(P):
            mu = P.mean(axis=0)
            C = (P - mu).T @ (P - mu) / len(P)
            lam, V = np.linalg.eigh(C)
            e = V[:, k] * np.sign(V[:, k] @ vref)
            return np.concatenate([e, mu])
        P0 = pts[ids].astype(np.float64)
        h = 1e-6
        ref = np.zeros((6, 6))
        for j in range(len(ids)):
            J = np.zeros((6, 3))
            for c in range(3):
                Pp, Pm = P0.copy(), P0.copy()
                Pp[j, c] += h
                Pm[j, c] -= h
                J[:, c] = (desc(Pp) - desc(Pm)) / (2 * h)
            Si = np.array([[c6[ids[j], 0], c6[ids[j], 1], c6[ids[j], 2]], [c6[ids[j], 1], c6[ids[j], 3], c6[ids[j], 4]],
                           [c6[ids[j], 2], c6[ids[j], 4], c6[ids[j], 5]]])
            ref += J @ Si @ J.T
        np.testing.assert_allclose(Sg[v], ref, rtol=1e-4, atol=1e-6 * np.abs(ref).max())


def test_anchored_model_scale_keeps_ratios_and_reduces_to_the_heuristic():
    """Eq. 4: the anchored model branch keeps the predicted axis ratios, puts the largest axis at
    d / f, and an isotropic prediction reproduces Eq. 6's size."""
    pts, _ = _cloud(7)
    vox = io.voxel_pca(pts, 5)
    nv = len(vox["n"])
    rng = np.random.default_rng(1)
    pred = np.concatenate([rng.uniform(-6, -1, (nv, 3)), rng.standard_normal((nv, 4)), rng.standard_normal((nv, 1))],
                          axis=1)
    pred[0, :3] = -3.0  # isotropic
    depth = rng.uniform(2, 20, len(pts))
    seg = np.zeros(len(pts), np.int64)
    a = io.cascade(pts, np.full((len(pts), 3), 0.5), depth, seg, vox, pred=pred, f=500.0, anchored=True)
    p = io.cascade(pts, np.full((len(pts), 3), 0.5), depth, seg, vox, pred=pred, f=500.0)
    m = a["branch"] == 0
    assert m.sum() > 100
    s, s0 = a["log_scales"][:, m], p["log_scales"][:, m]
    np.testing.assert_allclose(np.max(s, axis=0), np.log(depth[m] / 500.0), rtol=1e-12)
    np.testing.assert_allclose(s - s.max(axis=0), s0 - s0.max(axis=0), atol=1e-12)
    iso = m & (vox["voxel"] == 0)
    if iso.any():
        np.testing.assert_allclose(a["log_scales"][:, iso], np.tile(np.log(depth[iso] / 500.0), (3, 1)), rtol=1e-12)
