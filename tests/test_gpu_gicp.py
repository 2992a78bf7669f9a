"""GPU parity of the Gaussian-based loop registration (Sec. III-D, Eq. 13-16) against the FP64
oracle on the loop corridor: the source and target sets and the correspondences are integer
results (bit-exact); the normal equations and poses agree within float64 summation-order noise.

Workload: the loop corridor with 100k Gaussians; the source is the last segment (scans 190-199 m,
which close the loop), the target set is what the first four keyframes see within 30 m."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import synth
from oracle import gicp_oracle as go

pytestmark = pytest.mark.gpu

D_MAX, D_CORR = 30.0, 0.5
REL = 1e-9


@pytest.fixture(scope="module")
def scene():
    import paper_2604_12942_amd as gsr
    c = synth.config3(n_points=100_000)
    g = c["gaussians"]
    seg = c["segment_id"]
    cams = c["cameras"][:4]
    P = gsr.gaussians_to_device(g)
    return dict(g=g, seg=seg, src_seg=int(seg.max()), cams=cams, P=P, sh=g["sh_degree"],
                seg_d=torch.from_numpy(seg.astype(np.int32)).cuda(), cams_d=gsr.camera_tensor(cams))


def _oracle_sets(s):
    g = s["g"]
    src = np.nonzero(go.source_set(s["seg"], s["src_seg"]))[0]
    tgt = np.nonzero(go.target_set(g["means"], s["seg"], s["src_seg"], s["cams"], D_MAX))[0]
    cov = go.regularized_cov(g["quats"], g["log_scales"])
    return src, tgt, cov


def test_sets_bit_exact(scene):
    import paper_2604_12942_amd as gsr
    st = gsr.gicp_prepare(scene["P"], scene["sh"], scene["seg_d"], scene["src_seg"], scene["cams_d"], 4, D_MAX, D_CORR)
    torch.cuda.synchronize()
    ns, nt = [int(x) for x in st["counts"].cpu().numpy()]
    src, tgt, _ = _oracle_sets(scene)
    assert ns == src.size and nt == tgt.size and ns > 1000 and nt > 5000
    assert np.array_equal(st["src_index"][:ns].cpu().numpy(), src)
    assert np.array_equal(st["tgt_index"][:nt].cpu().numpy(), tgt)


def _pose(rotvec, t):
    R = Rotation.from_rotvec(rotvec).as_matrix()
    return R, np.asarray(t, np.float64)


def test_one_iteration_matches_oracle(scene):
    import paper_2604_12942_amd as gsr
    g = scene["g"]
    R0, t0 = _pose([0.004, -0.006, 0.012], [0.15, -0.1, 0.05])
    st = gsr.gicp_prepare(scene["P"], scene["sh"], scene["seg_d"], scene["src_seg"], scene["cams_d"], 4, D_MAX, D_CORR)
    pose = torch.tensor(np.concatenate([R0.ravel(), t0]), dtype=torch.float64, device="cuda")
    corr = torch.full((g["means"].shape[1],), -7, dtype=torch.int32, device="cuda")
    gsr.gicp_iterate(scene["P"], scene["sh"], st, pose, 1, corr=corr)
    torch.cuda.synchronize()
    src, tgt, cov = _oracle_sets(scene)
    ne = go.normal_equations(R0, t0, g["means"][:, src], cov[src], g["means"][:, tgt], cov[tgt], D_CORR)
    got_corr = corr[:src.size].cpu().numpy()
    assert np.array_equal(got_corr, ne["corr"]), int((got_corr != ne["corr"]).sum())
    stats = st["stats"].cpu().numpy()
    assert stats[29] == ne["count"] > 500
    iu = np.triu_indices(6)
    H = ne["H"][iu]
    assert np.all(np.abs(stats[:21] - H) <= REL * np.abs(ne["H"]).max())
    assert np.all(np.abs(stats[21:27] - ne["g"]) <= REL * np.abs(ne["g"]).max())
    assert abs(stats[27] - ne["cost"]) <= REL * ne["cost"] and abs(stats[28] - ne["sq"]) <= REL * ne["sq"]
    R1, t1, xi = go.gn_update(R0, t0, ne["H"], ne["g"])
    pz = pose.cpu().numpy()
    assert np.abs(stats[30:36] - xi).max() <= 1e-7 * np.abs(xi).max()
    assert np.abs(pz[:9] - R1.ravel()).max() < 1e-9 and np.abs(pz[9:] - t1).max() < 1e-9


def test_registration_converges_like_oracle(scene):
    from paper_2604_12942_amd import loop
    g = scene["g"]
    R0, t0 = _pose([0.0, 0.0, 0.015], [0.2, -0.15, 0.03])
    out = loop.register(scene["P"], scene["sh"], scene["seg_d"], scene["src_seg"], scene["cams_d"], 4, (R0, t0),
                        d_max=D_MAX, d_corr=D_CORR)
    src, tgt, cov = _oracle_sets(scene)
    ref = go.register(R0, t0, g["means"][:, src], cov[src], g["means"][:, tgt], cov[tgt], D_CORR)
    assert out["converged"] == ref["converged"] and out["accepted"] == ref["accepted"]
    assert out["converged"] and out["accepted"]
    assert abs(out["iterations"] - ref["iterations"]) <= 1
    assert np.abs(out["R"] - ref["R"]).max() < 1e-6 and np.abs(out["t"] - ref["t"]).max() < 1e-6
    # the map is consistent, so the loop correction is close to the identity
    assert np.abs(out["t"]).max() < 0.05 and np.abs(out["R"] - np.eye(3)).max() < 0.01


def test_too_few_correspondences_fail(scene):
    import paper_2604_12942_amd as gsr
    st = gsr.gicp_prepare(scene["P"], scene["sh"], scene["seg_d"], scene["src_seg"], scene["cams_d"], 4, D_MAX, D_CORR)
    far = torch.tensor(np.concatenate([np.eye(3).ravel(), [500.0, 0.0, 0.0]]), dtype=torch.float64, device="cuda")
    gsr.gicp_iterate(scene["P"], scene["sh"], st, far, 5)
    torch.cuda.synchronize()
    stats = st["stats"].cpu().numpy()
    assert stats[38] == 1.0 and stats[36] == 0.0 and stats[37] == 1.0
    assert np.array_equal(far.cpu().numpy()[9:], [500.0, 0.0, 0.0])


def test_transform_segment_and_cameras_match_oracle():
    import paper_2604_12942_amd as gsr
    rng = np.random.default_rng(9)
    n = 20_000
    g = synth.random_gaussians(6, n, 3)
    seg = rng.integers(0, 4, n).astype(np.int32)
    R, t = _pose([0.3, -0.2, 0.5], [1.0, -2.0, 0.5])
    P = gsr.gaussians_to_device(g)
    pose = torch.tensor(np.concatenate([R.ravel(), t]), dtype=torch.float64, device="cuda")
    gsr.transform_segment(P, 3, torch.from_numpy(seg).cuda(), 2, pose)
    cams = [synth.make_camera(_pose(rng.normal(0, 0.3, 3), [0, 0, 0])[0], rng.normal(0, 1, 3), 100, 100, 50, 40, 100, 80)
            for _ in range(3)]
    ct = gsr.camera_tensor(cams)
    gsr.transform_cameras(ct, 3, pose, mask=torch.tensor([1, 0, 1], dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    means, quats, sh = go.transform_segment(g, seg, 2, R, t)
    for name, exp in (("means", means), ("quats", quats), ("sh", sh)):
        got = P[name].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - exp) <= 2e-7 * np.abs(exp) + 1e-6 * np.abs(exp).max()), name
    for name in ("log_scales", "opacity_logits"):
        assert np.array_equal(P[name].cpu().numpy(), g[name].astype(np.float32)), name
    raw = ct.cpu().numpy().view(np.float32).reshape(3, 24)
    for k, cam in enumerate(cams):
        Rc, tc = go.transform_camera(cam, R, t) if k != 1 else (cam["R"].astype(np.float64), cam["t"].astype(np.float64))
        np.testing.assert_allclose(raw[k, :9], Rc.ravel(), atol=1e-6)
        np.testing.assert_allclose(raw[k, 9:12], tc, atol=1e-5)
