"""GPU parity of the supervision masks (Eq. 7) and the full loss (Eq. 9-12, masked L1 colour and
depth plus SSIM) against the FP64 oracle, alone and inside a differentiated render.

Masks and counts are integer results: bit-exact.  Loss values: 1e-5 relative.  Gradients:
|g - o| <= 1e-3 (|o| + rms(o)) per view and channel, the gradient tolerance of the rasterizer
(the float32 window moments lose about 1e-5 relative to cancellation in E[x^2] - mean^2)."""
import numpy as np
import pytest
import scipy.ndimage as nd
import torch

import oracle
import synth
from oracle import loss_oracle as lo

from gpu_common import grad_close, run_forward

pytestmark = pytest.mark.gpu


def _smooth_T(rng, V, H, W, k=9):
    T = np.stack([nd.uniform_filter(rng.random((H, W)), k) for _ in range(V)])
    T = (T - T.min()) / (T.max() - T.min())
    return T.astype(np.float32)


@pytest.mark.parametrize("tau,r", [(0.5, 0), (0.5, 2), (0.3, 5), (0.6, 8)])
def test_support_mask_bit_exact(tau, r):
    import paper_2604_12942_amd as gsr
    rng = np.random.default_rng(int(r * 10 + tau * 10))
    V, H, W = 4, 70, 100  # ragged against the 32 x 8 mask tile
    T = _smooth_T(rng, V, H, W)
    T[2] = 0.0  # fully supported view
    T[3] = 1.0  # unsupported view
    raster = gsr.Raster(W, H)
    mask, count = gsr.support_mask(torch.from_numpy(T).cuda(), V, raster, tau, r)
    torch.cuda.synchronize()
    got = mask.cpu().numpy().astype(bool)
    cnt = count.cpu().numpy().view(np.uint32)
    for v in range(V):
        _, exp = lo.support_masks(T[v], tau, r)
        assert np.array_equal(got[v], exp), (v, int((got[v] != exp).sum()))
        assert cnt[v] == exp.sum()
    assert cnt[3] == 0 and cnt[2] == (H - 2 * r) * (W - 2 * r)


def _loss_inputs(seed, V, S, H, W):
    rng = np.random.default_rng(seed)
    rgb = nd.gaussian_filter(rng.random((V, 3, H, W)), (0, 0, 1.5, 1.5)).astype(np.float32)
    trgb = np.clip(nd.gaussian_filter(rng.random((S, 3, H, W)), (0, 0, 1.0, 1.0))
                   + 0.1 * rng.standard_normal((S, 3, H, W)), 0, 1).astype(np.float32)
    dep = rng.uniform(2, 9, (V, H, W)).astype(np.float32)
    tdep = rng.uniform(2, 9, (S, H, W)).astype(np.float32)
    T = _smooth_T(rng, V, H, W)
    T[-1] = 1.0  # last view: empty mask
    idx = rng.permutation(S)[:V].astype(np.int32)
    return rgb, trgb, dep, tdep, T, idx


@pytest.mark.parametrize("lams,masked", [((0.8, 0.2, 0.2), True), ((1.0, 0.0, 0.2), True), ((0.8, 0.2, 0.0), False)])
def test_full_loss_matches_oracle(lams, masked):
    import paper_2604_12942_amd as gsr
    V, S, H, W = 3, 4, 72, 100  # 100 x 72: ragged against the 32 x 16 SSIM tile
    rgb, trgb, dep, tdep, T, idx = _loss_inputs(11, V, S, H, W)
    raster = gsr.Raster(W, H)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    mask = count = None
    if masked:
        mask, count = gsr.support_mask(t(T), V, raster, 0.5, 2)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gC = torch.full((V, 3, H, W), np.nan, device="cuda")
    gD = torch.full((V, H, W), np.nan, device="cuda")
    lr, ls, ld = lams
    gsr.loss(t(rgb), t(dep), t(trgb), t(tdep), V, raster, loss, gC, gD, mask=mask, count=count, lambda_rgb=lr,
             lambda_ssim=ls, lambda_depth=ld, target_index=t(idx))
    torch.cuda.synchronize()
    gC, gD = gC.cpu().numpy(), gD.cpu().numpy()
    exp_loss = 0.0
    for v in range(V):
        M = lo.support_masks(T[v], 0.5, 2)[1] if masked else None
        L, eC, eD = lo.masked_loss(rgb[v], dep[v], trgb[idx[v]], tdep[idx[v]], M, lr, ls, ld)
        exp_loss += L
        for c in range(3):
            bad = grad_close(gC[v, c], eC[c])
            assert bad.sum() == 0, (v, c, int(bad.sum()))
        assert grad_close(gD[v], eD).sum() == 0
        if masked and v == V - 1:
            assert not np.any(gC[v]) and not np.any(gD[v])
    assert abs(loss.item() - exp_loss) <= 1e-5 * abs(exp_loss), (loss.item(), exp_loss)


def test_masked_ssim_loss_through_the_renderer():
    """Render, mask from the render's own transmittance, full loss, backward to every parameter:
    against the oracle doing the same in FP64.  Gaussians that reach a knife-edge pixel's
    neighbourhood (erosion radius + two SSIM windows) are excluded, as in the rasterizer's parity."""
    import paper_2604_12942_amd as gsr
    g, cam = synth.config1()["gaussians"], synth.config1()["cameras"][0]
    W, H = int(cam["width"]), int(cam["height"])
    rng = np.random.default_rng(5)
    trgb = rng.uniform(0, 1, (1, 3, H, W)).astype(np.float32)
    tdep = rng.uniform(2, 10, (1, H, W)).astype(np.float32)
    o = oracle.render(g, cam)
    # threshold in the widest gap of the oracle's transmittance near 1/2 (no decision within the gap)
    Ts = np.sort(o["T"].ravel())
    mid = (Ts[:-1] + Ts[1:]) / 2
    gap = Ts[1:] - Ts[:-1]
    cand = np.abs(mid - 0.5) < 0.2
    k = np.argmax(np.where(cand, gap, -1))
    assert gap[k] > 2e-4, gap[k]
    tau = float(1.0 - mid[k])
    r_erode = 2
    M_o = lo.support_masks(o["T"].astype(np.float32), tau, r_erode)[1]
    L_o, eC, eD = lo.masked_loss(o["rgb"], o["depth"], trgb[0], tdep[0], M_o, 0.8, 0.2, 0.2)
    ob = oracle.render_bwd(g, cam, eC, eD)

    out, rast, P, ct = run_forward(g, [cam])
    mask, count = gsr.support_mask(rast.T_final, 1, rast.raster, tau, r_erode)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gC = torch.empty(1, 3, H, W, device="cuda")
    gD = torch.empty(1, H, W, device="cuda")
    gsr.loss(rast.rgb, rast.depth, torch.from_numpy(trgb).cuda(), torch.from_numpy(tdep).cuda(), 1, rast.raster, loss,
             gC, gD, mask=mask, count=count, lambda_rgb=0.8, lambda_ssim=0.2, lambda_depth=0.2)
    grads = {k: torch.zeros_like(P[k]) for k in gsr.PARAM_NAMES}
    rast.backward(P, g["sh_degree"], ct, gC, gD, grads)
    torch.cuda.synchronize()

    knife = ob["knife_px"]
    # dL/dC(q) reads the images within 10 pixels of q (two window passes) and the mask there,
    # which reads the transmittance within r_erode of it
    reach = r_erode + 10
    near = nd.binary_dilation(knife, structure=np.ones((2 * reach + 1,) * 2, bool)) if knife.any() else knife
    M_g = mask.cpu().numpy()[0].astype(bool)
    assert np.array_equal(M_g[~near], M_o[~near])
    keep = ~ob["knife_g"]
    if near.any():
        ys, xs = np.nonzero(near)
        for ids in oracle.contributors(g, cam, np.stack([xs, ys], 1)):
            keep[ids] = False
    else:
        assert abs(loss.item() - L_o) <= 1e-5 * abs(L_o)
    assert keep.mean() > 0.5
    for k in gsr.PARAM_NAMES:
        bad = grad_close(grads[k].cpu().numpy(), ob[k], mask=keep)
        assert bad.sum() == 0, (k, int(bad.sum()))


def test_full_loss_headline_size():
    """The full loss in the timed step's configuration: 8 views of 1280x720 in one launch, the
    support mask (tau_geo 0.5, erosion radius 2) and lambda = (0.8, 0.2, 0.2).  Every gradient
    pixel of two views against the oracle; the last view's mask is empty, so its gradients are
    exactly zero."""
    import paper_2604_12942_amd as gsr
    V, S, H, W = 8, 16, 720, 1280
    rgb, trgb, dep, tdep, T, idx = _loss_inputs(12, V, S, H, W)
    raster = gsr.Raster(W, H, 8, 32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    mask, count = gsr.support_mask(t(T), V, raster, 0.5, 2)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gC = torch.full((V, 3, H, W), np.nan, device="cuda")
    gD = torch.full((V, H, W), np.nan, device="cuda")
    gsr.loss(t(rgb), t(dep), t(trgb), t(tdep), V, raster, loss, gC, gD, mask=mask, count=count, lambda_rgb=0.8,
             lambda_ssim=0.2, lambda_depth=0.2, target_index=t(idx))
    torch.cuda.synchronize()
    gC, gD = gC.cpu().numpy(), gD.cpu().numpy()
    assert np.isfinite(loss.item()) and np.all(np.isfinite(gC)) and np.all(np.isfinite(gD))
    for v in (0, 3):
        M = lo.support_masks(T[v], 0.5, 2)[1]
        assert 0 < M.sum() < M.size
        _, eC, eD = lo.masked_loss(rgb[v], dep[v], trgb[idx[v]], tdep[idx[v]], M, 0.8, 0.2, 0.2)
        for c in range(3):
            bad = grad_close(gC[v, c], eC[c])
            assert bad.sum() == 0, (v, c, int(bad.sum()))
        assert grad_close(gD[v], eD).sum() == 0, v
    assert not np.any(gC[V - 1]) and not np.any(gD[V - 1])
