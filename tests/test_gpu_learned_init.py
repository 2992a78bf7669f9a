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
