"""GPU tests of the learned-init pipeline: per-voxel training targets against the oracle's
definition on seeded synthetic Gaussians, the cascade over a scene, and network training that
lowers the loss."""
import numpy as np
import pytest
import torch

import synth
from oracle import init_oracle as io
from oracle import pointnet_oracle as pn

pytestmark = pytest.mark.gpu


def _scene(seed=300):
    c = synth.c5_scene(seed, n_points=30000, targets=False)
    return c


def test_voxel_targets_match_oracle():
    from paper_2604_12942_amd import learned_init as li
    c = _scene()
    sc = li.SceneInit(c["points"], c["colors"], c["depth"], c["segment"], c["n_segments"], seed=4)
    n = sc.n
    rng = np.random.default_rng(0)
    ls = rng.uniform(-4, -1, (3, n)).astype(np.float32)
    q = rng.standard_normal((4, n)).astype(np.float32)
    lo = rng.standard_normal(n).astype(np.float32)
    P = dict(log_scales=torch.from_numpy(ls).cuda(), quats=torch.from_numpy(q).cuda(),
             opacity_logits=torch.from_numpy(lo).cuda())
    cov_t, o_t, has = sc.targets(P)
    torch.cuda.synchronize()
    o = io.voxel_pca(c["points"], 4)
    ct, ot, hs = pn.targets_from_gaussians(o, ls.astype(np.float64), q.astype(np.float64), lo.astype(np.float64),
                                           np.arange(n))
    nv = len(o["n"])
    assert int(sc.vox["n_voxels"].item()) == nv
    assert np.array_equal(has[:nv].cpu().numpy().astype(bool), hs)
    six = np.stack([ct[:, 0, 0], ct[:, 0, 1], ct[:, 0, 2], ct[:, 1, 1], ct[:, 1, 2], ct[:, 2, 2]])
    got = cov_t[:, :nv].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - six) <= 1e-5 * (np.abs(six) + np.abs(six).max(axis=0, keepdims=True)))
    np.testing.assert_allclose(o_t[:nv].cpu().numpy(), ot, rtol=1e-5, atol=1e-6)


def test_network_training_lowers_the_loss():
    from paper_2604_12942_amd import learned_init as li
    c = _scene(301)
    sc = li.SceneInit(c["points"], c["colors"], c["depth"], c["segment"], c["n_segments"], seed=1)
    P, br = sc.gaussians(beta=0.7)
    tg = sc.targets(P)
    w = li.init_weights(3)
    first = li.train_pointnet([sc], [tg], w, 1)
    last = li.train_pointnet([sc], [tg], w, 60)
    assert np.isfinite(last) and last < 0.5 * first
    P2, br2 = sc.gaussians(weights=w)
    b = br2.cpu().numpy()
    assert np.all(b <= 2) and np.any(b == 0)


def _psnr_run(c, P, iters, seed, every=50):
    """Optimise P on the scene's training views; held-out PSNR every `every` iterations."""
    import paper_2604_12942_amd as gsr
    from paper_2604_12942_amd.optimize import MapOptimizer
    cams = c["cameras"]
    W, H = cams[0]["width"], cams[0]["height"]
    raster = gsr.Raster(W, H, 16, 16)
    tv, hv = c["train_views"], c["held_out"]
    trgb = torch.from_numpy(np.stack([c["targets"][k][0] for k in tv])).cuda()
    tdep = torch.from_numpy(np.stack([c["targets"][k][1] for k in tv])).cuda()
    hrgb = torch.from_numpy(np.stack([c["targets"][k][0] for k in hv])).cuda()
    opt = MapOptimizer(P, 3, gsr.camera_tensor([cams[k] for k in tv]), trgb, tdep, raster, 4, lambda_depth=0.2)
    held = gsr.Rasterizer(P["means"].shape[1], len(hv), raster)
    hcams = gsr.camera_tensor([cams[k] for k in hv])
    rng = np.random.default_rng(seed)

    def psnr():
        rgb, _, _ = held.forward(P, 3, hcams)
        return float(10 * torch.log10(1.0 / torch.mean((rgb.clamp(0, 1) - hrgb) ** 2)).item())

    out = [(0, psnr())]
    for it in range(iters):
        opt.set_views(rng.choice(len(tv), 4, replace=False))
        opt.step()
        if (it + 1) % every == 0:
            out.append((it + 1, psnr()))
    return out


def test_learned_init_gain_over_voxel_pca():
    """What the trained network adds to the cascade (Eq. 3) on held-out scenes: the network is
    trained on maps the plain optimiser produced from the voxel-PCA init of training scenes, then
    both inits of each test scene start identical optimisers.  The learned init starts with a
    higher held-out PSNR on every test scene; the iterations each needs to reach the PCA run's
    final PSNR less 0.25 dB are printed (on these scenes the PCA init gets there first: the gain
    is in the starting quality, not in the iterations to the target)."""
    from paper_2604_12942_amd import learned_init as li
    train = [synth.c5_scene(400 + k, n_points=30000, n_keyframes=12) for k in range(4)]
    test = [synth.c5_scene(500 + k, n_points=30000, n_keyframes=12) for k in range(2)]
    scenes, targets = [], []
    for k, c in enumerate(train):
        sc = li.SceneInit(c["points"], c["colors"], c["depth"], c["segment"], c["n_segments"], seed=k)
        P, _ = sc.gaussians(beta=1.0)
        _psnr_run(c, P, 800, k, every=800)
        scenes.append(sc)
        targets.append(sc.targets(P))
    w = li.init_weights(0)
    li.train_pointnet(scenes, targets, w, 300)
    for k, c in enumerate(test):
        sc = li.SceneInit(c["points"], c["colors"], c["depth"], c["segment"], c["n_segments"], seed=10 + k)
        PA, _ = sc.gaussians(beta=1.0)
        PB, br = sc.gaussians(weights=w)
        assert np.any(br.cpu().numpy() == 0)
        ca = _psnr_run(c, PA, 800, 100 + k)
        cb = _psnr_run(c, PB, 800, 100 + k)
        target = ca[-1][1] - 0.25
        first = lambda cur: next((i for i, p in cur if p >= target), None)
        print("test scene %d: PSNR pca %s learned %s; iterations to %.2f dB: pca %s learned %s"
              % (k, [round(p, 2) for _, p in ca], [round(p, 2) for _, p in cb], target, first(ca), first(cb)))
        assert cb[0][1] > ca[0][1] + 1.0, (ca[0], cb[0])
