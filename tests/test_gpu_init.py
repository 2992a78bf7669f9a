"""GPU parity of the initialisation path against the FP64 oracle: voxel binning and point selection
(bit-exact), voxel PCA (moments, eigensystem, canonical frame, class, reliability) and the
cascade's per-point branch and parameters."""
import numpy as np
import pytest
import torch

import synth
from oracle import init_oracle as io

pytestmark = pytest.mark.gpu


def _room_points(n, seed=1):
    scene = synth.room_scene(seed)
    rng = np.random.default_rng(seed + 1)
    scans = rng.uniform(-15.0, 15.0, (4, 2))
    pts, surf, nrm, rngs, scan = scene.lidar(rng, scans, int(n * 2.5))
    keep = np.sort(rng.choice(pts.shape[0], n, replace=False))
    return pts[keep].astype(np.float32), scene.albedo(pts[keep], surf[keep]).astype(np.float32), \
        rngs[keep].astype(np.float32), (scan[keep] % 3).astype(np.int32)


def _packed(key):
    k = np.asarray(key, np.int64)
    return ((k[:, 0] + 1024) << 21) | ((k[:, 1] + 1024) << 10) | (k[:, 2] + 511)


def _run(pts, seed):
    import paper_2604_12942_amd as gsr
    t = torch.from_numpy(np.ascontiguousarray(pts.T)).cuda()
    out = gsr.voxel_pca(t, seed)
    torch.cuda.synchronize()
    return t, out


def _margins_ok(o):
    """Voxels whose discrete decisions (class, reliability) are far from their thresholds."""
    lam = o["evals"]
    ok = np.abs(lam[:, 0] / io.TAU_P - 1) > 1e-4
    with np.errstate(divide="ignore", invalid="ignore"):
        ok &= ~(np.abs((lam[:, 2] / lam[:, 0]) / io.TAU_L - 1) <= 1e-4)
        ok &= ~np.isfinite(o["trace"]) | (np.abs(o["trace"] / io.REL_TRACE - 1) > 1e-4)
    return ok


def _frame_ok(o):
    """Voxels whose canonical frame is unique and stable: distinct eigenvalues and an
    unambiguous largest component in every column."""
    lam = o["evals"]
    gaps = np.min(np.diff(lam, axis=1), axis=1) / np.maximum(lam[:, 2], 1e-30)
    ok = (gaps > 1e-3) & (o["n"] >= 3)
    R = o["R"]
    for j in range(3):
        a = np.sort(np.abs(R[:, :, j]), axis=1)
        ok &= (a[:, 2] - a[:, 1]) > 1e-3
    return ok


@pytest.mark.parametrize("n,seed", [(40000, 7), (6000, 123456789012345)])
def test_voxel_pca_matches_oracle(n, seed):
    pts, col, rng_, seg = _room_points(n)
    t, out = _run(pts, seed)
    o = io.voxel_pca(pts, seed)
    nv = int(out["n_voxels"].item())
    assert nv == len(o["n"]) and int(out["n_outside"].item()) == 0
    key = out["key"][:nv].cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(key, _packed(o["key"]))
    cnt = out["count"][:nv].cpu().numpy().astype(np.int64)
    assert np.array_equal(cnt, o["n_all"])
    start = out["start"][:nv].cpu().numpy().astype(np.int64)
    order = out["point_order"][:n].cpu().numpy().astype(np.int64)
    for v in range(nv):
        assert np.array_equal(order[start[v]:start[v] + min(cnt[v], 32)], o["ids"][v]), v
    assert np.array_equal(out["point_voxel"][:n].cpu().numpy().astype(np.int64), o["voxel"])
    mu = out["mu"][:, :nv].cpu().numpy().T.astype(np.float64)
    np.testing.assert_allclose(mu, o["mu"], rtol=0, atol=2e-6 * np.abs(o["mu"]).max())
    lam = out["evals"][:, :nv].cpu().numpy().T.astype(np.float64)
    sc = o["evals"][:, 2:3] + 1e-12
    assert np.all(np.abs(lam - o["evals"]) <= 1e-5 * sc + 1e-12)
    ok = _margins_ok(o)
    assert ok.mean() > 0.98
    fr = _frame_ok(o)
    assert fr.sum() >= 100
    R = out["R"][:, :nv].cpu().numpy().T.reshape(nv, 3, 3).astype(np.float64)
    assert np.all(np.abs(R[fr] - o["R"][fr]) <= 1e-3)
    s = out["s_pca"][:, :nv].cpu().numpy().T.astype(np.float64)
    assert np.all(np.abs(s - o["s_pca"]) <= 1e-4)
    cls = out["cls"][:nv].cpu().numpy()
    rel = out["reliable"][:nv].cpu().numpy().astype(bool)
    assert np.array_equal(cls[ok], o["cls"][ok])
    assert np.array_equal(rel[ok], o["reliable"][ok])
    tr = out["trace"][:nv].cpu().numpy().astype(np.float64)
    fin = np.isfinite(o["trace"]) & ok
    np.testing.assert_allclose(tr[fin], o["trace"][fin], rtol=1e-4)
    assert np.all(~np.isfinite(tr[ok & ~np.isfinite(o["trace"])]))
    # every class occurs in a LiDAR room scene
    assert set(np.unique(cls)) >= {0, 2}


def test_voxel_pca_outside_points_and_tiny_inputs():
    rng = np.random.default_rng(3)
    pts = rng.uniform(-2, 2, (500, 3)).astype(np.float32)
    pts[:7, 0] = 600.0  # beyond the key range in x
    t, out = _run(pts, 5)
    assert int(out["n_outside"].item()) == 7
    pv = out["point_voxel"][:500].cpu().numpy().view(np.uint32)
    assert np.all(pv[:7] == 0xFFFFFFFF)
    o = io.voxel_pca(pts[7:], 5)
    assert int(out["n_voxels"].item()) == len(o["n"])
    t1, out1 = _run(pts[7:8], 1)
    assert int(out1["n_voxels"].item()) == 1 and out1["cls"][0].item() == io.UNRELIABLE


@pytest.mark.parametrize("with_model,anchored", [(False, False), (True, False), (True, True)])
def test_cascade_matches_oracle(with_model, anchored):
    import paper_2604_12942_amd as gsr
    n = 20000
    pts, col, rng_, seg = _room_points(n, seed=2)
    t, vox = _run(pts, 11)
    o = io.voxel_pca(pts, 11)
    nv = len(o["n"])
    pred = None
    pred_t = None
    if with_model:
        r = np.random.default_rng(9)
        pred = np.concatenate([r.uniform(np.log(0.001), np.log(0.3), (nv, 3)), r.standard_normal((nv, 4)),
                               r.standard_normal((nv, 1))], axis=1)
        pred[r.random(nv) < 0.1, 0] = np.nan
        pt = np.zeros((8, n), np.float32)
        pt[:, :nv] = pred.T
        pred_t = torch.from_numpy(pt).cuda()
    c_t = torch.from_numpy(np.ascontiguousarray(col.T)).cuda()
    d_t = torch.from_numpy(rng_).cuda()
    s_t = torch.from_numpy(seg).cuda()
    P, br = gsr.cascade(t, c_t, d_t, vox, pred=pred_t, focal=640.0, beta=0.0, segment=s_t, n_segments=3, sh_degree=1,
                        anchored=anchored)
    torch.cuda.synchronize()
    g = io.cascade(pts, col, rng_, seg, o, pred=pred, f=640.0, sh_degree=1, anchored=anchored)
    ok = _margins_ok(o)[o["voxel"]]
    if with_model:
        # a prediction near the validity bounds is a knife edge in float32
        s = pred[:, :3]
        edge = np.any((np.abs(s - np.log(0.002)) < 1e-5) | (np.abs(s - np.log(0.5)) < 1e-5), axis=1)
        ok &= ~edge[o["voxel"]]
    b = br.cpu().numpy()
    assert np.array_equal(b[ok], g["branch"][ok])
    assert set(np.unique(g["branch"])) >= ({0, 1, 2} if with_model else {1, 2})
    for k in ("means", "log_scales", "opacity_logits", "sh"):
        got = P[k].cpu().numpy().astype(np.float64)
        exp = g[k]
        assert np.all(np.abs(got[..., ok] - exp[..., ok]) <= 1e-5 * (np.abs(exp[..., ok]) + 1)), k
    # quaternions: the same rotation (sign fixed by w >= 0) where the PCA frame is unique
    q = P["quats"].cpu().numpy().astype(np.float64)
    qok = ok & ((g["branch"] != 1) | _frame_ok(o)[o["voxel"]])
    assert np.all(np.abs(q[:, qok] - g["quats"][:, qok]) <= 1e-3)


def test_voxel_pca_with_point_covariances_matches_oracle():
    """Eq. 1-2 with anisotropic LiDAR point covariances: the full descriptor covariance, its
    direction trace and the reliability flags against the oracle's per-point sum."""
    import paper_2604_12942_amd as gsr
    n, seed = 40000, 11
    scene = synth.room_scene(1)
    rng = np.random.default_rng(2)
    scans = rng.uniform(-15.0, 15.0, (4, 2))
    pts, surf, nrm, rngs, scan = scene.lidar(rng, scans, int(n * 2.5))
    keep = np.sort(rng.choice(pts.shape[0], n, replace=False))
    pts = pts[keep].astype(np.float32)
    org = np.c_[scans[scan[keep]], np.full(n, 1.8)]
    cov = synth.lidar_point_cov(pts, org)
    t = torch.from_numpy(np.ascontiguousarray(pts.T)).cuda()
    out = gsr.voxel_pca(t, seed, point_cov=torch.from_numpy(np.ascontiguousarray(cov.T)).cuda(), sigma_g=True)
    torch.cuda.synchronize()
    o = io.voxel_pca(pts, seed)
    Sg, tr_o, rel_o = io.descriptor_covariance(pts, o, cov)
    nv = len(o["n"])
    assert int(out["n_voxels"].item()) == nv
    o2 = dict(o, trace=tr_o)
    ok = _margins_ok(o2)
    assert ok.mean() > 0.98
    rel = out["reliable"][:nv].cpu().numpy().astype(bool)
    assert np.array_equal(rel[ok], rel_o[ok])
    assert rel_o.sum() > 50 and (~rel_o & (o["cls"] != io.UNRELIABLE)).sum() > 0
    tr = out["trace"][:nv].cpu().numpy().astype(np.float64)
    fin = np.isfinite(tr_o) & ok
    np.testing.assert_allclose(tr[fin], tr_o[fin], rtol=1e-4)
    # full covariance on voxels with a unique frame (the cross block follows v_k's sign)
    sel = fin & _frame_ok(o)
    assert sel.sum() > 50
    g = out["sigma_g"][:, :nv].cpu().numpy().T.astype(np.float64)
    iu = np.triu_indices(6)
    exp = Sg[:, iu[0], iu[1]]
    diag = Sg[:, np.arange(6), np.arange(6)]
    scale = np.sqrt(diag[:, iu[0]] * diag[:, iu[1]])
    bad = np.abs(g[sel] - exp[sel]) > 1e-4 * scale[sel] + 1e-12
    assert bad.sum() == 0, np.argwhere(bad)[:5]
    assert not g[o["cls"] == io.UNRELIABLE].any()


def test_cascade_validity_bounds_match_oracle():
    """Predictions exactly at the float32 log-scale bounds (valid) and one float32 step outside
    them (invalid) take the oracle's branch: the bound test is inclusive and taken in float32."""
    import paper_2604_12942_amd as gsr
    n = 6000
    pts, col, rng_, seg = _room_points(n, seed=3)
    t, vox = _run(pts, 5)
    o = io.voxel_pca(pts, 5)
    nv = len(o["n"])
    lo32, hi32 = np.float32(np.log(0.002)), np.float32(np.log(0.5))
    edge = [lo32, np.nextafter(lo32, np.float32(-np.inf)), hi32, np.nextafter(hi32, np.float32(np.inf)),
            np.nextafter(lo32, np.float32(0)), np.nextafter(hi32, np.float32(-1))]
    pred = np.zeros((nv, 8), np.float32)
    pred[:, :3] = np.log(0.05)
    pred[:, 3] = 1.0
    for v in range(nv):
        pred[v, v % 3] = edge[v % len(edge)]
    pred[5::11, 3:7] = 0.0  # zero quaternions
    pt = np.zeros((8, n), np.float32)
    pt[:, :nv] = pred.T
    P, br = gsr.cascade(t, torch.from_numpy(np.ascontiguousarray(col.T)).cuda(), torch.from_numpy(rng_).cuda(), vox,
                        pred=torch.from_numpy(pt).cuda(), focal=640.0, beta=0.0,
                        segment=torch.from_numpy(seg).cuda(), n_segments=3, sh_degree=0)
    torch.cuda.synchronize()
    g = io.cascade(pts, col, rng_, seg, o, pred=pred.astype(np.float64), f=640.0, sh_degree=0)
    valid = io.prediction_valid(pred.astype(np.float64))
    assert valid.sum() > 0 and (~valid).sum() > 0
    b = br.cpu().numpy()
    assert np.array_equal(b == 0, valid[o["voxel"]])
    ok = _margins_ok(o)[o["voxel"]]
    assert np.array_equal(b[ok], g["branch"][ok])
