"""Pins of the oracle's hand-derived backward (every parameter and the camera pose).

  * FP64 central finite differences with h = 1e-6 on a 5k-Gaussian SH-degree-3 scene at
    160x120 with a random pose (all 6 pose components + 300 stratified parameter scalars);
    a sample whose +-h renders differ in any discrete decision is redrawn.
  * invariants: translation gauge sum_i dL/dmu_i = R^T dL/drho; <dL/dq_i, q_i> = 0; the
    rotation gauge at SH degree 0; permutation invariance of the image.
  * a dense torch float64 autograd formulation of the same function on <= 8 Gaussians
    (library autodiff, independent of the hand derivation).
  * sparse Adam against torch.optim.Adam / SparseAdam.
"""
import math

import numpy as np
import pytest
import torch

import synth

PARAMS = ("means", "log_scales", "quats", "opacity_logits", "sh")


def upstream(cam, seed=11):
    rng = np.random.default_rng(seed)
    H, W = cam["height"], cam["width"]
    return rng.standard_normal((3, H, W)), rng.standard_normal((H, W))


def lin_loss(orc, g, cam, GC, GD):
    r = orc.render(g, cam)
    return float(np.sum(GC * r["rgb"]) + np.sum(GD * r["depth"])), r


def fd_of(rp, rm, GC, GD, h):
    # difference the images first: pixels the perturbation does not reach cancel exactly
    return float(np.sum(GC * (rp["rgb"] - rm["rgb"])) + np.sum(GD * (rp["depth"] - rm["depth"]))) / (2 * h)


def f64(g):
    out = {k: np.array(g[k], np.float64) for k in PARAMS}
    out["sh_degree"] = g["sh_degree"]
    return out


def perturb_pose(cam, k, h):
    c = dict(cam)
    R = np.asarray(cam["R"], np.float64)
    t = np.asarray(cam["t"], np.float64)
    if k < 3:
        t = t.copy()
        t[k] += h
    else:
        w = np.zeros(3)
        w[k - 3] = h
        Kx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        th = np.linalg.norm(w)
        Rot = np.eye(3) + math.sin(th) / th * Kx + (1 - math.cos(th)) / th ** 2 * Kx @ Kx
        R = Rot @ R
        t = Rot @ t
    c["R"], c["t"] = R, t
    return c


@pytest.fixture(scope="module")
def c4a():
    c = synth.config4a()
    cam = dict(c["cameras"][0])
    # the camera centre is -R^T t, which is the true centre only for an orthogonal R: use the
    # float64 polar factor of the float32 rotation so the gauge identities hold to rounding
    U, _, Vt = np.linalg.svd(np.asarray(cam["R"], np.float64))
    cam["R"] = U @ Vt
    return f64(c["gaussians"]), cam


def test_finite_differences_config4a(orc, c4a):
    g, cam = c4a
    GC, GD = upstream(cam)
    an = orc.render_bwd(g, cam, GC, GD)
    base = orc.render(g, cam)
    assert base["n"].max() > 5
    h = 1e-6
    rng = np.random.default_rng(123)
    n = g["means"].shape[1]
    vis = np.nonzero((an["screen"] != 0).any(1) & ~an["knife_g"])[0]
    checks = []
    # stratified parameter samples: 60 per parameter tensor
    for name in PARAMS:
        rows = g[name].shape[0] if g[name].ndim == 2 else 1
        got = 0
        tries = 0
        while got < 60 and tries < 400:
            tries += 1
            i = int(rng.choice(vis))
            r = int(rng.integers(rows))
            gp, gm = f64(g), f64(g)
            if g[name].ndim == 2:
                gp[name][r, i] += h
                gm[name][r, i] -= h
                a = an[name][r, i]
            else:
                gp[name][i] += h
                gm[name][i] -= h
                a = an[name][i]
            rp, rm = orc.render(gp, cam), orc.render(gm, cam)
            if not (np.array_equal(rp["n"], base["n"]) and np.array_equal(rm["n"], base["n"])):
                continue  # a discrete decision moved: redraw
            checks.append((name, fd_of(rp, rm, GC, GD, h), a))
            got += 1
        assert got == 60, name
    # the pose moves every Gaussian, so some pixel of 19,200 may flip a decision within +-h:
    # such pixels (and knife edges) are masked out of the upstream gradient on both sides
    for k in range(6):
        rp = orc.render(g, perturb_pose(cam, k, h))
        rm = orc.render(g, perturb_pose(cam, k, -h))
        keep = (rp["n"] == base["n"]) & (rm["n"] == base["n"]) & (base["margin"] >= 1e-5)
        assert keep.mean() > 0.99
        GCk, GDk = GC * keep, GD * keep
        ank = orc.render_bwd(g, cam, GCk, GDk)["pose"][k] if not keep.all() else an["pose"][k]
        checks.append(("pose%d" % k, fd_of(rp, rm, GCk, GDk, h), ank))
    # floor: float64 rounding of the two renders (~1e-16 relative per pixel, a few hundred
    # changed pixels) divided by 2h
    bad = [(nm, fd, a) for nm, fd, a in checks if abs(fd - a) > 1e-4 * abs(a) + 1e-8]
    assert not bad, bad[:10]
    assert len(checks) == 306


def test_translation_gauge_and_quaternion_orthogonality(orc, c4a):
    g, cam = c4a
    GC, GD = upstream(cam, 12)
    an = orc.render_bwd(g, cam, GC, GD)
    R = np.asarray(cam["R"], np.float64)
    # a joint shift of every mean and the camera centre leaves the image unchanged
    lhs = an["means"].sum(1)
    rhs = R.T @ an["pose"][:3]
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-10 * np.abs(rhs).max())
    # the quaternion is normalised, so its gradient is orthogonal to it
    dots = np.sum(an["quats"] * g["quats"], axis=0)
    scale = np.linalg.norm(an["quats"], axis=0) * np.linalg.norm(g["quats"], axis=0) + 1e-300
    assert np.max(np.abs(dots) / scale) < 1e-10


def test_rotation_gauge_sh0(orc):
    # At SH degree 0 a joint world rotation of means, orientations and camera leaves the image
    # unchanged: sum_i [mu_i x dL/dmu_i + (quaternion term)] + R^T (t x dL/drho - dL/dphi) = 0.
    c = synth.config1()
    g = f64(c["gaussians"])
    U, _, Vt = np.linalg.svd(synth.small_rotation(np.random.default_rng(9), 8.0))
    cam = synth.make_camera(np.eye(3), [0.1, -0.1, 0.2], 100.0, 100.0, 64.0, 48.0, 128, 96)
    cam["R"] = U @ Vt  # exactly orthogonal in float64
    GC, GD = upstream(cam, 13)
    an = orc.render_bwd(g, cam, GC, GD)
    mu = g["means"]
    q = g["quats"]
    tot = np.cross(mu.T, an["means"].T).sum(0)
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        # d/dw_k of (1, w/2) (x) q  = 1/2 (0, e_k) (x) q
        qv = q[1:]
        dq0 = -0.5 * (e @ qv)
        dqv = 0.5 * (q[0][None, :] * e[:, None] + np.cross(e, qv.T).T)
        tot[k] += np.sum(an["quats"][0] * dq0) + np.sum(an["quats"][1:] * dqv)
    R = np.asarray(cam["R"], np.float64)
    t = np.asarray(cam["t"], np.float64)
    # the camera follows as R' = R Rot^T, t' = t, i.e. the left perturbation phi = -R w,
    # rho = (R w) x t
    tot += R.T @ np.cross(t, an["pose"][:3]) - R.T @ an["pose"][3:]
    ref = np.abs(np.cross(mu.T, an["means"].T)).sum(0).max()
    assert np.abs(tot).max() < 1e-10 * ref
    # and the forward is invariant to the joint rotation
    w = np.array([0.02, -0.03, 0.015])
    Kx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    th = np.linalg.norm(w)
    Rot = np.eye(3) + math.sin(th) / th * Kx + (1 - math.cos(th)) / th ** 2 * Kx @ Kx
    g2 = f64(g)
    g2["means"] = Rot @ mu
    qw = np.array([math.cos(th / 2), *(math.sin(th / 2) * w / th)])
    a0, av = qw[0], qw[1:]
    g2["quats"] = np.vstack([a0 * q[0] - av @ q[1:], a0 * q[1:] + q[0][None, :] * av[:, None] + np.cross(av, q[1:].T).T])
    cam2 = dict(cam)
    cam2["R"] = R @ Rot.T
    r1 = orc.render(g, cam)
    r2 = orc.render(g2, cam2)
    np.testing.assert_allclose(r2["rgb"], r1["rgb"], atol=1e-9)


def test_permutation_invariance(orc):
    c = synth.config1()
    g = f64(c["gaussians"])
    cam = c["cameras"][0]
    perm = np.random.default_rng(4).permutation(g["means"].shape[1])
    gp = {k: (g[k][..., perm]) for k in PARAMS}
    gp["sh_degree"] = g["sh_degree"]
    a = orc.render(g, cam)
    b = orc.render(gp, cam)
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["depth"], b["depth"])
    GC, GD = upstream(cam, 3)
    ga = orc.render_bwd(g, cam, GC, GD)
    gb = orc.render_bwd(gp, cam, GC, GD)
    np.testing.assert_allclose(gb["means"], ga["means"][:, perm], rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------------------------------
# dense torch float64 autograd formulation (decisions taken from a detached forward)
# ------------------------------------------------------------------------------------------

def _sh_torch(d, degree):
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    Y = [torch.full_like(x, 0.5 / math.sqrt(pi))]
    if degree >= 1:
        c1 = math.sqrt(3 / (4 * pi))
        Y += [c1 * y, c1 * z, c1 * x]
    if degree >= 2:
        a = 0.5 * math.sqrt(15 / pi)
        Y += [a * x * y, a * y * z, 0.25 * math.sqrt(5 / pi) * (3 * z * z - 1), a * x * z,
              0.25 * math.sqrt(15 / pi) * (x * x - y * y)]
    if degree >= 3:
        b = 0.25 * math.sqrt(35 / (2 * pi))
        c = 0.25 * math.sqrt(21 / (2 * pi))
        Y += [b * y * (3 * x * x - y * y), 0.5 * math.sqrt(105 / pi) * x * y * z, c * y * (5 * z * z - 1),
              0.25 * math.sqrt(7 / pi) * z * (5 * z * z - 3), c * x * (5 * z * z - 1),
              0.25 * math.sqrt(105 / pi) * z * (x * x - y * y), b * x * (x * x - 3 * y * y)]
    return torch.stack(Y, 1)  # [n, K]


def torch_render(P, cam, degree, xi):
    """Dense differentiable render (all pixels x all Gaussians) following the same definitions."""
    R0 = torch.tensor(np.asarray(cam["R"], np.float64))
    t0 = torch.tensor(np.asarray(cam["t"], np.float64))
    rho, phi = xi[:3], xi[3:]
    zero = torch.zeros((), dtype=torch.float64)
    Kx = torch.stack([torch.stack([zero, -phi[2], phi[1]]), torch.stack([phi[2], zero, -phi[0]]),
                      torch.stack([-phi[1], phi[0], zero])])
    E = torch.linalg.matrix_exp(Kx)
    R = E @ R0
    t = E @ t0 + rho
    fx, fy, cx, cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    W, H = cam["width"], cam["height"]
    mu = P["means"].T  # [n,3]
    p = mu @ R.T + t
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    q = P["quats"].T
    q = q / q.norm(dim=1, keepdim=True)
    w_, a_, b_, c_ = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    Rq = torch.stack([torch.stack([1 - 2 * (b_ * b_ + c_ * c_), 2 * (a_ * b_ - w_ * c_), 2 * (a_ * c_ + w_ * b_)], 1),
                      torch.stack([2 * (a_ * b_ + w_ * c_), 1 - 2 * (a_ * a_ + c_ * c_), 2 * (b_ * c_ - w_ * a_)], 1),
                      torch.stack([2 * (a_ * c_ - w_ * b_), 2 * (b_ * c_ + w_ * a_), 1 - 2 * (a_ * a_ + b_ * b_)], 1)], 1)
    M = Rq * torch.exp(P["log_scales"].T)[:, None, :]
    Sig = M @ M.transpose(1, 2)
    Sc = R @ Sig @ R.T
    limx, limy = 1.3 * W / (2 * fx), 1.3 * H / (2 * fy)
    tx = torch.clamp(x / z, -limx, limx)
    ty = torch.clamp(y / z, -limy, limy)
    zeros = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zeros, -fx * tx / z], 1), torch.stack([zeros, fy / z, -fy * ty / z], 1)], 1)
    Sp = J @ Sc @ J.transpose(1, 2) + 0.3 * torch.eye(2, dtype=torch.float64)
    Q = torch.linalg.inv(Sp)
    u = fx * x / z + cx
    v = fy * y / z + cy
    o = torch.sigmoid(P["opacity_logits"])
    Cc = -R.T @ t
    dv = mu - Cc
    d = dv / dv.norm(dim=1, keepdim=True)
    Y = _sh_torch(d, degree)
    K = Y.shape[1]
    sh = P["sh"].T.reshape(-1, K, 3)
    pre = (Y[:, :, None] * sh).sum(1) + 0.5
    rgb = torch.clamp(pre, min=0.0)
    jj, ii = torch.meshgrid(torch.arange(H, dtype=torch.float64), torch.arange(W, dtype=torch.float64), indexing="ij")
    dx = (ii.reshape(-1, 1) + 0.5) - u[None, :]
    dy = (jj.reshape(-1, 1) + 0.5) - v[None, :]
    m = Q[:, 0, 0] * dx * dx + 2 * Q[:, 0, 1] * dx * dy + Q[:, 1, 1] * dy * dy
    ar = o[None, :] * torch.exp(-0.5 * m)
    ok = (ar >= 1 / 255).detach() & (z > cam["z_near"]).detach()[None, :]
    a = torch.where(ok, torch.clamp(ar, max=0.99), torch.zeros_like(ar))
    order = torch.argsort(z.detach(), stable=True)  # (z, index) order; no ties in these draws
    a = a[:, order]
    one_m = 1 - a
    Tprefix = torch.cumprod(torch.cat([torch.ones_like(a[:, :1]), one_m], 1), 1)  # T before k, and after all
    # termination: first k with T_before_k * (1 - a_k) < 1e-4 is not composited, nor later ones
    stop = (Tprefix[:, 1:] < 1e-4).detach()
    keep = torch.cumsum(stop.to(torch.int64), 1) == 0
    a = torch.where(keep, a, torch.zeros_like(a))
    T = torch.cumprod(torch.cat([torch.ones_like(a[:, :1]), 1 - a], 1), 1)
    wgt = a * T[:, :-1]
    col = wgt @ rgb[order]
    dep = wgt @ z[order]
    Tf = T[:, -1]
    bg = torch.tensor(np.asarray(cam["bg"], np.float64))
    col = col + Tf[:, None] * bg[None, :]
    return col.T.reshape(3, H, W), dep.reshape(H, W)


@pytest.mark.parametrize("degree,seed", [(0, 21), (3, 22), (3, 23)])
def test_oracle_backward_matches_torch_autograd(orc, degree, seed):
    g = synth.random_gaussians(seed, 8, degree, xy_half=0.4, z_range=(2.0, 3.0), log_scale_mean=-2.3,
                               log_scale_std=0.4)
    g = f64(g)
    g["opacity_logits"] = g["opacity_logits"] + 1.5  # make stacking and termination likely
    rng = np.random.default_rng(seed)
    cam = synth.make_camera(synth.small_rotation(rng, 6.0), rng.uniform(-0.05, 0.05, 3), 30.0, 30.0, 8.0, 8.0,
                            16, 16, bg=(0.1, 0.2, 0.3))
    GC, GD = upstream(cam, seed)
    an = orc.render_bwd(g, cam, GC, GD)
    ref = orc.render(g, cam)
    assert an["n_knife"] == 0
    P = {k: torch.tensor(g[k], requires_grad=True) for k in PARAMS}
    xi = torch.zeros(6, dtype=torch.float64, requires_grad=True)
    col, dep = torch_render(P, cam, degree, xi)
    np.testing.assert_allclose(col.detach().numpy(), ref["rgb"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(dep.detach().numpy(), ref["depth"], rtol=1e-12, atol=1e-13)
    L = (col * torch.tensor(GC)).sum() + (dep * torch.tensor(GD)).sum()
    L.backward()
    for k in PARAMS:
        np.testing.assert_allclose(an[k], P[k].grad.numpy(), rtol=1e-9, atol=1e-11, err_msg=k)
    np.testing.assert_allclose(an["pose"], xi.grad.numpy(), rtol=1e-9, atol=1e-11)


def test_adam_matches_torch(orc):
    rng = np.random.default_rng(8)
    rows, cols = 37, 5
    p0 = rng.standard_normal((cols, rows))
    grads = [rng.standard_normal((cols, rows)) * 1e-3 for _ in range(4)]
    tp = torch.tensor(p0.T.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for s, gr in enumerate(grads, 1):
        p, _, m, v = orc.adam(p, gr.copy(), m, v, None, 1e-2, step=s)
        opt.zero_grad()
        tp.grad = torch.tensor(gr.T.copy())
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy().T, rtol=1e-13, atol=1e-15)


def test_sparse_adam_masked_rows_match_sparse_adam(orc):
    rng = np.random.default_rng(9)
    rows, cols = 23, 3
    p0 = rng.standard_normal((cols, rows))
    tp = torch.tensor(p0.T.copy(), requires_grad=True)
    opt = torch.optim.SparseAdam([tp], lr=5e-3, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for s in range(1, 5):
        mask = rng.uniform(size=rows) < 0.6
        gr = rng.standard_normal((cols, rows)) * np.where(mask, 1.0, 0.0)[None, :]
        p, g_after, m, v = orc.adam(p, gr.copy(), m, v, mask.astype(np.uint8), 5e-3, step=s)
        assert np.all(g_after == 0)
        idx = np.nonzero(mask)[0]
        tp.grad = torch.sparse_coo_tensor(torch.tensor(idx)[None, :], torch.tensor(gr.T[idx].copy()), (rows, cols))
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy().T, rtol=1e-12, atol=1e-14)
