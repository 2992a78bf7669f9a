"""Depth slices of long tiles (gsr_render_fwd_sliced): the front-to-back recurrence of Eq. 8
regrouped by the associativity of the transmittance product, checked against the FP64 oracle
and against the whole-tile forward on a vanishing-point pile-up whose central tiles hold about
11,000 instances (tiles above 8192 are cut into slices of 1024), with pixels that terminate in a
middle slice and pixels that walk every slice.  Tolerances and knife-edge exclusion as in the other parity tests."""
import numpy as np
import pytest
import torch

import oracle

from gpu_common import GRAD_RTOL, KNIFE, grad_close, img_close, long_tile_scene, run_forward

pytestmark = pytest.mark.gpu

SLICE = 1024
SPLIT_MIN = 8192
G, CAM = long_tile_scene()
_CACHE = {}


def _oracle():
    if "o" not in _CACHE:
        _CACHE["o"] = oracle.render(G, CAM)
    return _CACHE["o"]


def _lengths(rast):
    rg = rast.tile_ranges.cpu().numpy().view(np.uint32).astype(np.int64).reshape(-1, 2)
    return rg[:, 1] - rg[:, 0]


@pytest.mark.parametrize("tile", [(16, 16), (8, 32), (32, 8)])
def test_sliced_forward_matches_oracle(tile):
    out, rast, P, ct = run_forward(G, [CAM], tile=tile)
    ln = _lengths(rast)
    assert (ln > SPLIT_MIN).sum() >= 2  # the path under test is taken
    o = _oracle()
    ok = o["margin"] >= KNIFE
    assert (~ok).sum() <= 0.01 * ok.size
    m3 = np.broadcast_to(ok, o["rgb"].shape)
    assert img_close(out["rgb"][0], o["rgb"], mask=m3).sum() == 0
    assert img_close(out["depth"][0], o["depth"], mask=ok).sum() == 0
    assert img_close(1 - out["T"][0], o["alpha"], mask=ok).sum() == 0
    # walks that end in a later slice, terminated or not
    assert (out["last"][0] > SLICE).sum() > 100
    assert ((out["last"][0] > SLICE) & (out["T"][0] < 1e-3)).sum() > 10


def test_sliced_forward_matches_whole_tiles():
    a, ra, *_ = run_forward(G, [CAM], sliced=False)
    b, rb, *_ = run_forward(G, [CAM], sliced=True)
    ok = _oracle()["margin"] >= KNIFE
    assert img_close(b["rgb"][0], a["rgb"][0], mask=np.broadcast_to(ok, a["rgb"][0].shape)).sum() == 0
    assert img_close(b["depth"][0], a["depth"][0], mask=ok).sum() == 0
    assert img_close(b["T"][0], a["T"][0], mask=ok).sum() == 0
    assert np.array_equal(b["last"][0][ok], a["last"][0][ok])
    # tiles of at most 8192 instances are composited by the same code from the same start
    ln = _lengths(rb)
    short = np.zeros(ok.shape, bool)
    T = rb.raster.tiles
    for t in np.nonzero(ln[:T] <= SPLIT_MIN)[0]:
        ty, tx = divmod(int(t), rb.raster.ntx)
        short[ty * rb.raster.tile_h:(ty + 1) * rb.raster.tile_h, tx * rb.raster.tile_w:(tx + 1) * rb.raster.tile_w] = True
    assert short.any() and (~short).any()
    assert np.array_equal(b["rgb"][0][:, short], a["rgb"][0][:, short])
    assert np.array_equal(b["T"][0][short], a["T"][0][short])


def test_backward_after_sliced_forward_matches_oracle():
    import paper_2604_12942_amd as gsr
    out, rast, P, ct = run_forward(G, [CAM])
    rng = np.random.default_rng(5)
    H, W = CAM["height"], CAM["width"]
    GC = rng.standard_normal((3, H, W)).astype(np.float32)
    GD = rng.standard_normal((H, W)).astype(np.float32)
    o = oracle.render_bwd(G, CAM, GC.astype(np.float64), GD.astype(np.float64), want_pose=False)
    grads = {k: torch.zeros_like(P[k]) for k in gsr.PARAM_NAMES}
    rast.backward(P, G["sh_degree"], ct, torch.from_numpy(GC[None]).cuda(), torch.from_numpy(GD[None]).cuda(), grads)
    torch.cuda.synchronize()
    keep = ~o["knife_g"]
    assert keep.mean() > 0.85  # faint Gaussians near the 1/255 cut-off make many knife-edge candidates
    for k in gsr.PARAM_NAMES:
        gk = grads[k].cpu().numpy().astype(np.float64)
        bad = grad_close(gk, o[k], mask=keep)
        assert bad.sum() == 0, (k, bad.sum())


def test_slice_list_overflow_leaves_tiles_whole():
    """A slice workspace sized for too small an instance capacity cannot hold the long tiles'
    slices: those tiles are composited whole, exactly as by the whole-tile forward."""
    import paper_2604_12942_amd as gsr
    a, ra, *_ = run_forward(G, [CAM], sliced=False)
    ws = torch.empty(gsr.render_fwd_sliced_workspace(1, ra.raster, 1), dtype=torch.uint8, device="cuda")
    ct = gsr.camera_tensor([CAM])
    gsr.render_fwd(ra.splats, ra.inst_gid, ra.tile_ranges, ct, 1, ra.raster, ra.rgb, ra.depth, ra.T_final, ra.last,
                   tile_order=ra.tile_order, ws=ws, capacity=1)
    torch.cuda.synchronize()
    assert np.array_equal(ra.rgb.cpu().numpy().astype(np.float64), a["rgb"])
    assert np.array_equal(ra.T_final.cpu().numpy().astype(np.float64), a["T"])
    assert np.array_equal(ra.last.cpu().numpy(), a["last"])


def test_sliced_forward_two_views():
    """Two views in one launch, the pile-up seen head-on and from the side: each view's long
    tiles are sliced independently and both images match the whole-tile forward."""
    from scipy.spatial.transform import Rotation
    import synth
    cam2 = synth.make_camera(Rotation.from_rotvec([0.0, 0.25, 0.0]).as_matrix(), np.array([0.5, 0.0, 0.3]),
                             60.0, 60.0, 32.0, 32.0, 64, 64)
    a, ra, *_ = run_forward(G, [CAM, cam2], sliced=False)
    b, rb, *_ = run_forward(G, [CAM, cam2], sliced=True)
    assert (_lengths(rb) > SPLIT_MIN).sum() >= 2
    for v in range(2):
        o = oracle.render(G, [CAM, cam2][v])
        ok = o["margin"] >= KNIFE
        assert img_close(b["rgb"][v], a["rgb"][v], mask=np.broadcast_to(ok, a["rgb"][v].shape)).sum() == 0
        assert img_close(b["T"][v], a["T"][v], mask=ok).sum() == 0
        assert np.array_equal(b["last"][v][ok], a["last"][v][ok])


def _one_tile_scene(n, opaque_front, seed=21):
    """n small Gaussians inside one 16x16 tile (a 16x16 image, f = 16), each within 3 pixels of
    the centre so that every one reaches only that tile, at distinct depths 2-8 m, faint (opacity
    0.01) so that the walk reaches the back of the list; with opaque_front, 40 nearly opaque
    ones lie at 2.0-2.1 m, so that most pixels terminate inside the first slice."""
    rng = np.random.default_rng(seed)
    f, W = 16.0, 16
    z = rng.permutation(np.linspace(2.0, 8.0, n))
    px = rng.uniform(5.0, 11.0, (2, n))
    means = np.stack([(px[0] - W / 2) * z / f, (px[1] - W / 2) * z / f, z])
    log_scales = np.log(np.full((3, n), 0.7) * z / f)
    logit = np.full(n, np.log(0.01 / 0.99))
    if opaque_front:
        k = 40
        z2 = np.linspace(2.0, 2.1, k)
        p2 = rng.uniform(4.0, 12.0, (2, k))
        means[:, :k] = np.stack([(p2[0] - W / 2) * z2 / f, (p2[1] - W / 2) * z2 / f, z2])
        log_scales[:, :k] = np.log(np.full((3, k), 2.5) * z2 / f)
        logit[:k] = 6.0
    quats = np.zeros((4, n))
    quats[0] = 1.0
    sh = rng.standard_normal((3, n))
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    g = dict(means=f32(means), log_scales=f32(log_scales), quats=f32(quats), opacity_logits=f32(logit), sh=f32(sh),
             sh_degree=0)
    import synth
    cam = synth.make_camera(np.eye(3), np.zeros(3), f, f, W / 2.0, W / 2.0, W, W)
    return g, cam


@pytest.mark.parametrize("opaque_front", [False, True])
def test_slice_boundary_backward(opaque_front):
    """A tile one instance above the split (8193: nine slices, the last holding one instance) runs
    the L1 backward in the forward's slices (gsr_render_bwd_l1 given the sliced forward's
    workspace): records equal the whole-tile backward's to float rounding and the forward the
    oracle; with an opaque front most pixels terminate in the first slice, so the eight slices
    behind it must leave zero records."""
    import paper_2604_12942_amd as gsr
    n = SPLIT_MIN + 1
    g, cam = _one_tile_scene(n, opaque_front)
    out, rast, P, ct = run_forward(g, [cam])
    assert _lengths(rast)[0] == n, _lengths(rast)[0]
    o = oracle.render(g, cam)
    ok = o["margin"] >= KNIFE
    assert img_close(out["rgb"][0], o["rgb"], mask=np.broadcast_to(ok, o["rgb"].shape)).sum() == 0
    assert img_close(1 - out["T"][0], o["alpha"], mask=ok).sum() == 0
    if opaque_front:
        assert (out["last"][0] <= SLICE).mean() > 0.5
    else:
        assert (out["last"][0] > 8 * SLICE).sum() > 0  # pixels that reach the one-instance slice
    rng = np.random.default_rng(3)
    trgb = torch.from_numpy(rng.uniform(0, 1, (1, 3, 16, 16)).astype(np.float32)).cuda()
    tdep = torch.from_numpy(rng.uniform(2, 8, (1, 16, 16)).astype(np.float32)).cuda()
    ws = torch.empty((gsr.render_bwd_l1_workspace(1, rast.raster) + 255) // 256 * 64, dtype=torch.int32, device="cuda")
    recs = {}
    for sliced in (False, True):
        rast.forward(P, g["sh_degree"], ct, sliced=sliced)
        rast.dinst.fill_(-7)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        gsr.render_bwd_l1(rast.splats, rast.inst_gid, rast.inst_emit, rast.tile_ranges, ct, 1, rast.raster, rast.rgb,
                          rast.depth, rast.T_final, rast.last, trgb, tdep, 0.2, loss, rast.dinst, ws,
                          tile_order=rast.tile_order, fwd_ws=rast.fwd_ws if sliced else None, capacity=rast.capacity)
        torch.cuda.synchronize()
        recs[sliced] = (rast.screen_grads().cpu().numpy().astype(np.float64).reshape(-1, 10), loss.item())
    a, la = recs[False]
    b, lb = recs[True]
    assert abs(la - lb) <= 1e-6 * abs(la)
    rms = np.sqrt(np.mean(a ** 2, axis=0))
    assert np.all(np.abs(b - a) <= 1e-4 * (np.abs(a) + rms))
    if opaque_front:
        # Gaussians behind every pixel's last contributor get exactly zero
        last_max = int(out["last"][0].max())
        order = rast.inst_gid.cpu().numpy()[:n]
        behind = order[last_max:]
        assert behind.size > 0 and np.all(a[behind] == 0) and np.all(b[behind] == 0)
