"""Pins of the point-network oracle: BF16 rounding against torch's bfloat16 conversion, the
forward and backward against torch autograd on the same rounded tensors (straight-through at the
rounding points), the loss gradient against finite differences, and the closed forms KL = 0 at
the target and permutation invariance of the max-pool."""
import numpy as np
import pytest
import torch

from oracle import pointnet_oracle as pn


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -1 - 2 ** -8, 0.0, 65504.0]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(pn.bf16(x), ref)
    assert pn.bf16(np.array([1 + 2 ** -8]))[0] == 1.0            # tie to even
    assert pn.bf16(np.array([1 + 3 * 2 ** -9]))[0] == 1 + 2 ** -7


def _inputs(seed, nv=6):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((nv, pn.ROWS, 3)) * 0.4
    F = rng.standard_normal((nv, pn.N_FEAT))
    W = pn.init_weights(seed)
    for k in ("b1", "b2", "b3", "b4", "b5"):
        W[k] = (rng.standard_normal(W[k].shape) * 0.1).astype(np.float32)
    A = rng.standard_normal((nv, 3, 3)) * 0.05
    cov = A @ np.transpose(A, (0, 2, 1)) + np.eye(3) * 1e-3
    o = rng.uniform(0.05, 0.95, nv)
    return W, X, F, cov, o


def _torch_forward(W, X, F):
    """Same network in torch float64 with straight-through BF16 rounding."""
    def rnd(t):
        return t + (torch.from_numpy(pn.bf16(t.detach().numpy())) - t).detach()
    Wt = {k: torch.tensor(np.asarray(v, np.float64), requires_grad=True) for k, v in W.items()}
    Wr = {k: rnd(Wt[k]) if k.startswith("W") else Wt[k] for k in Wt}
    x = rnd(torch.from_numpy(X))
    h1 = rnd(torch.relu(x @ Wr["W1"] + Wr["b1"]))
    h2 = rnd(torch.relu(h1 @ Wr["W2"] + Wr["b2"]))
    h3 = torch.relu(h2 @ Wr["W3"] + Wr["b3"])
    g = h3.max(dim=1).values
    z = rnd(torch.cat([g, torch.from_numpy(F)], dim=1))
    h4 = rnd(torch.relu(z @ Wr["W4"] + Wr["b4"]))
    return h4 @ Wr["W5"] + Wr["b5"], Wt


def test_forward_and_backward_match_torch_autograd():
    W, X, F, cov, o = _inputs(1)
    y, keep = pn.forward(W, X, F, keep=True)
    yt, Wt = _torch_forward(W, X, F)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    L, dy = pn.loss(y, cov, o)
    G = pn.backward(W, keep, dy, round_grads=False)
    yt.backward(torch.from_numpy(dy))
    for k in W:
        np.testing.assert_allclose(G[k], Wt[k].grad.numpy(), rtol=1e-9, atol=1e-12, err_msg=k)


def test_loss_gradient_matches_finite_differences():
    W, X, F, cov, o = _inputs(2)
    y = pn.forward(W, X, F)
    y[:, 3:7] += 0.3  # away from a degenerate quaternion
    y[:, :3] = 0.1 * y[:, :3] + np.log(0.06)  # scales comparable to the targets: KL of order one
    L, dy = pn.loss(y, cov, o)
    h = 1e-6
    for i in range(y.shape[0]):
        for j in range(8):
            yp, ym = y.copy(), y.copy()
            yp[i, j] += h
            ym[i, j] -= h
            fd = (pn.loss(yp, cov, o)[0] - pn.loss(ym, cov, o)[0]) / (2 * h)
            assert abs(fd - dy[i, j]) <= 1e-6 * abs(dy[i, j]) + 1e-9, (i, j, fd, dy[i, j])


def test_kl_vanishes_at_the_target_and_pool_is_permutation_invariant():
    rng = np.random.default_rng(3)
    q = rng.standard_normal((5, 4))
    s = rng.uniform(-3, -1, (5, 3))
    R = pn.quat_to_rot(q / np.linalg.norm(q, axis=1, keepdims=True))
    cov = R @ (np.exp(2 * s)[:, :, None] * np.transpose(R, (0, 2, 1)))
    o = rng.uniform(0.1, 0.9, 5)
    y = np.concatenate([s, q * 2.5, np.log(o / (1 - o))[:, None]], axis=1)
    L, dy = pn.loss(y, cov, o)
    assert abs(L) < 1e-12 and np.abs(dy[:, :7]).max() < 1e-12
    W, X, F, _, _ = _inputs(4)
    perm = rng.permutation(pn.ROWS)
    np.testing.assert_array_equal(pn.forward(W, X, F), pn.forward(W, X[:, perm], F))


def test_rounded_backward_stays_close_to_exact():
    W, X, F, cov, o = _inputs(5, nv=40)
    y, keep = pn.forward(W, X, F, keep=True)
    _, dy = pn.loss(y, cov, o)
    Ge = pn.backward(W, keep, dy, round_grads=False)
    Gr = pn.backward(W, keep, dy, round_grads=True)
    for k in W:
        scale = np.abs(Ge[k]).max() + 1e-30
        assert np.abs(Gr[k] - Ge[k]).max() <= 2e-2 * scale, k


def test_knife_screen_flags_a_rounding_midpoint_and_nothing_without_jitter():
    """The BF16 knife-edge screen: with zero jitter nothing moves; a first-layer activation placed
    exactly on a BF16 rounding midpoint (1 + 2^-8) moves the outputs that depend on it."""
    W, X, F, cov, o = _inputs(6, nv=3)
    ys, gs = pn.knife_spread(W, X, F, realisations=3, seed=0, cov_t=cov, o_t=o)
    assert ys.shape == (3, 8) and set(gs) == set(W)
    zero = pn.Jitter(0, c=0.0)
    y0 = pn.forward(W, X, F)
    np.testing.assert_array_equal(pn.forward(W, X, F, jitter=zero), y0)
    W2 = {k: v.copy() for k, v in W.items()}
    X2 = np.zeros_like(X)
    X2[0, :, 0] = 1.0                     # voxel 0: every row is (1, 0, 0)
    W2["W1"][:, 0] = [1.0, 0.0, 0.0]
    W2["b1"][0] = 2.0 ** -8               # a1[..., 0] = 1 + 2^-8: a BF16 midpoint
    _, keep = pn.forward(W2, X2, F, keep=True)
    assert np.all(keep["a1"][0, :, 0] == 1.0 + 2.0 ** -8)
    spread, _ = pn.knife_spread(W2, X2, F, realisations=8, seed=1)
    assert spread[0].max() > 0.0
