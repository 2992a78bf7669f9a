"""GPU tests of the optimisation step: the fused projection-backward + sparse Adam entry point
against the separate project_bwd + adam_step path (same gradients, same update), and the
sparse-update semantics (only visible Gaussians of unfrozen segments move)."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _opt(fused, g, cams, tgt_rgb, tgt_dep, seg, min_seg, **kw):
    import paper_2604_12942_amd as gsr
    from paper_2604_12942_amd.optimize import MapOptimizer
    P = gsr.gaussians_to_device(g)
    raster = gsr.Raster(cams[0]["width"], cams[0]["height"])
    pool = gsr.camera_tensor(cams)
    return MapOptimizer(P, g["sh_degree"], pool, tgt_rgb, tgt_dep, raster, len(cams), segment_id=seg,
                        min_segment=min_seg, fused=fused, **kw)


def test_fused_step_equals_separate_step():
    c = synth.config4a()
    g = c["gaussians"]
    rng = np.random.default_rng(0)
    cams = [c["cameras"][0]]
    for k in range(2):
        cams.append(synth.make_camera(synth.small_rotation(rng, 8.0), rng.uniform(-0.2, 0.2, 3), 125.0, 125.0, 80.0,
                                      60.0, 160, 120))
    H, W = 120, 160
    trgb = torch.from_numpy(rng.uniform(0, 1, (3, 3, H, W)).astype(np.float32)).cuda()
    tdep = torch.from_numpy(rng.uniform(2, 10, (3, H, W)).astype(np.float32)).cuda()
    n = g["means"].shape[1]
    seg = torch.from_numpy((np.arange(n) % 4).astype(np.int32)).cuda()
    a = _opt(True, g, cams, trgb, tdep, seg, 2)
    b = _opt(False, g, cams, trgb, tdep, seg, 2)
    before = {k: a.P[k].clone() for k in a.P if k != "sh_degree"}
    for step in range(3):
        for o in (a, b):
            o.set_views([0, 1, 2] if step % 2 == 0 else [2, 0, 1])
            o.step()
    torch.cuda.synchronize()
    # the two paths compute the same gradients (each from its own render backward, whose LDS
    # adds come in run-dependent order); the update is compared to rounding raised by Adam's
    # normalisation, the moments relative to their rms
    for k in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        pa, pb = a.P[k].cpu().numpy(), b.P[k].cpu().numpy()
        assert np.allclose(pa, pb, rtol=2e-6, atol=1e-6), k
        ma, mb = a.m[k].cpu().numpy().astype(np.float64), b.m[k].cpu().numpy().astype(np.float64)
        rms = np.sqrt(np.mean(mb ** 2))
        assert np.all(np.abs(ma - mb) <= 1e-4 * (np.abs(mb) + rms)), k
        # frozen segments (0, 1) and never-visible rows keep their values exactly
        moved = np.any(pa != before[k].cpu().numpy(), axis=0) if pa.ndim == 2 else pa != before[k].cpu().numpy()
        segs = np.arange(n) % 4
        assert not np.any(moved[segs < 2]), k
        assert np.any(moved[segs >= 2]), k


FULL_LOSS = dict(lambda_rgb=0.8, lambda_ssim=0.2, support=(0.5, 2))


@pytest.mark.parametrize("full", [False, True])
def test_graph_replay_matches_eager_step(full):
    """The fused step captured into HIP graphs (cut before the render backward) and replayed,
    with eager work and synchronisations between replays, follows the eager step; also with the
    support mask and the SSIM term in the loss."""
    c = synth.config4a()
    g = c["gaussians"]
    rng = np.random.default_rng(2)
    cams = [c["cameras"][0]]
    for k in range(2):
        cams.append(synth.make_camera(synth.small_rotation(rng, 8.0), rng.uniform(-0.2, 0.2, 3), 125.0, 125.0, 80.0,
                                      60.0, 160, 120))
    H, W = 120, 160
    trgb = torch.from_numpy(rng.uniform(0, 1, (3, 3, H, W)).astype(np.float32)).cuda()
    tdep = torch.from_numpy(rng.uniform(2, 10, (3, H, W)).astype(np.float32)).cuda()
    kw = FULL_LOSS if full else {}
    a = _opt(True, g, cams, trgb, tdep, None, 0, **kw)
    b = _opt(True, g, cams, trgb, tdep, None, 0, **kw)
    views = [[0, 1, 2], [2, 0, 1], [1, 2, 0], [0, 2, 1], [2, 1, 0]]
    for o in (a, b):
        o.set_views(views[0])
        o.step()
    b.capture(split=("render_bwd",))
    assert len(b.graphs) == 2
    for k in range(1, len(views)):
        a.set_views(views[k])
        la = float(a.step().item())
        b.set_views(views[k])
        lb = float(b.replay().item())
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum().item()  # eager work between replays
        assert np.isfinite(junk)
        assert abs(la - lb) <= 1e-6 * abs(la), (k, la, lb)
        # the render backward's four waves add to a Gaussian's LDS accumulators in run-dependent
        # order, so two runs of the same step agree to float rounding, which Adam's
        # normalisation raises to a few 1e-7 on parameters whose gradient nearly cancels
        for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            pa, pb = a.P[name].cpu().numpy(), b.P[name].cpu().numpy()
            assert np.allclose(pa, pb, rtol=2e-6, atol=1e-6), (k, name)
    assert int(b.step_dev.item()) == len(views)


def _three_views(seed):
    c = synth.config4a()
    rng = np.random.default_rng(seed)
    cams = [c["cameras"][0]]
    for k in range(2):
        cams.append(synth.make_camera(synth.small_rotation(rng, 8.0), rng.uniform(-0.2, 0.2, 3), 125.0, 125.0, 80.0,
                                      60.0, 160, 120))
    H, W = 120, 160
    trgb = torch.from_numpy(rng.uniform(0, 1, (3, 3, H, W)).astype(np.float32)).cuda()
    tdep = torch.from_numpy(rng.uniform(2, 10, (3, H, W)).astype(np.float32)).cuda()
    return c["gaussians"], cams, trgb, tdep


def test_overflowed_bin_sort_changes_nothing():
    """A bin/sort whose instances exceed the capacity empties its frame: no visible pair, empty
    tile ranges, no emitted pair; the render is background and the fused backward + Adam step
    leaves every parameter, moment and pose gradient untouched."""
    import paper_2604_12942_amd as gsr
    g, cams, trgb, tdep = _three_views(4)
    o = _opt(True, g, cams, trgb, tdep, None, 0)
    o.set_views([0, 1, 2])
    o.step()  # sizes the buffers
    torch.cuda.synchronize()
    r = o.rast
    need = r.instances()
    r._alloc_instances(need // 2)
    before = {k: o.P[k].clone() for k in gsr.PARAM_NAMES}
    m_before = {k: o.m[k].clone() for k in gsr.PARAM_NAMES}
    o.set_views([1, 2, 0])
    o.step(check_capacity=False)
    torch.cuda.synchronize()
    assert r.overflowed() and r.instances() > r.capacity
    assert torch.count_nonzero(r.tile_info.view(4, -1)[0]).item() == 0
    assert torch.count_nonzero(r.tile_ranges).item() == 0
    assert int(r.n_pairs.item()) == 0
    assert torch.all(r.T_final == 1.0).item() and torch.count_nonzero(r.rgb).item() == 0
    assert int(o.vis_count.item()) == 0 and torch.count_nonzero(o.row_mask).item() == 0
    assert torch.count_nonzero(r.dpose).item() == 0
    for k in gsr.PARAM_NAMES:
        assert torch.equal(o.P[k], before[k]) and torch.equal(o.m[k], m_before[k]), k


def test_replay_regrows_an_overflowed_capacity():
    """A captured step whose view set needs more instances than the captured capacity is
    detected after the replay, captured again with room and run again: the result follows the
    eager optimiser that never overflowed."""
    g, cams, trgb, tdep = _three_views(5)
    a = _opt(True, g, cams, trgb, tdep, None, 0)
    b = _opt(True, g, cams, trgb, tdep, None, 0)
    views = [[0, 1, 2], [2, 0, 1], [1, 2, 0]]
    for o in (a, b):
        o.set_views(views[0])
        o.step()
    torch.cuda.synchronize()
    b.rast._alloc_instances(b.rast.instances() // 2)
    small = b.rast.capacity
    b.capture(split=("render_bwd",))
    for k in range(1, len(views)):
        a.set_views(views[k])
        la = float(a.step().item())
        b.set_views(views[k])
        lb = float(b.replay().item())
        torch.cuda.synchronize()
        assert abs(la - lb) <= 1e-6 * abs(la), (k, la, lb)
    assert b.rast.capacity > small and not b.overflowed()
    assert int(b.step_dev.item()) == len(views) == int(a.step_dev.item())
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        pa, pb = a.P[name].cpu().numpy(), b.P[name].cpu().numpy()
        assert np.allclose(pa, pb, rtol=2e-6, atol=1e-6), name


@pytest.mark.parametrize("scene", ["three_views", "pile_up"])
def test_fused_render_step_equals_separate_launches(scene):
    """gsr_render_step (one persistent launch) and gsr_render_bwd_l1 (the loss inside the render
    backward) against gsr_render_fwd_sliced + gsr_loss_l1 + gsr_render_bwd: images and last
    positions bit for bit, the loss to float64 summation order, the per-pair screen-space gradients
    to the float rounding of the backward's LDS sums; the pile-up has tiles long enough to be
    composited in depth slices (finished by the workgroup that completes their last slice)."""
    import paper_2604_12942_amd as gsr
    from gpu_common import long_tile_scene
    if scene == "three_views":
        g, cams, _, _ = _three_views(6)
    else:
        g, cam = long_tile_scene()
        cams = [cam, synth.make_camera(synth.small_rotation(np.random.default_rng(1), 3.0), np.zeros(3), 60.0, 60.0,
                                       32.0, 32.0, 64, 64)]
    V = len(cams)
    H, W = cams[0]["height"], cams[0]["width"]
    rng = np.random.default_rng(11)
    trgb = torch.from_numpy(rng.uniform(0, 1, (V, 3, H, W)).astype(np.float32)).cuda()
    tdep = torch.from_numpy(rng.uniform(2, 10, (V, H, W)).astype(np.float32)).cuda()
    raster = gsr.Raster(W, H, 16, 16)
    P = gsr.gaussians_to_device(g)
    ct = gsr.camera_tensor(cams)
    r = gsr.Rasterizer(P["means"].shape[1], V, raster)
    r.forward(P, g["sh_degree"], ct, sliced=True)
    loss_a = torch.zeros(1, dtype=torch.float64, device="cuda")
    gC = torch.empty(V, 3, H, W, device="cuda")
    gD = torch.empty(V, H, W, device="cuda")
    gsr.loss_l1(r.rgb, r.depth, trgb, tdep, V, raster, 0.2, loss_a, gC, gD)
    r.render_backward(ct, gC, gD)
    torch.cuda.synchronize()
    ref = dict(rgb=r.rgb.clone(), depth=r.depth.clone(), T=r.T_final.clone(), last=r.last.clone())
    ds_a = r.screen_grads().cpu().numpy().astype(np.float64)
    if scene == "pile_up":
        lens = (r.tile_ranges.view(-1, 2)[:, 1] - r.tile_ranges.view(-1, 2)[:, 0]).cpu().numpy()
        assert lens.max() > 8192, lens.max()
    for k in (r.rgb, r.depth, r.T_final, r.last, r.dinst):
        k.fill_(-7)
    loss_b = torch.zeros(1, dtype=torch.float64, device="cuda")
    gsr.render_step(r.splats, r.inst_gid, r.inst_emit, r.tile_ranges, ct, V, raster, trgb, tdep, 0.2, r.rgb,
                    r.depth, r.T_final, r.last, loss_b, r.dinst, r.capacity, r.fwd_ws, tile_order=r.tile_order)
    torch.cuda.synchronize()
    assert torch.equal(r.rgb, ref["rgb"]) and torch.equal(r.depth, ref["depth"])
    assert torch.equal(r.T_final, ref["T"]) and torch.equal(r.last, ref["last"])
    assert abs(loss_a.item() - loss_b.item()) <= 1e-12 * abs(loss_a.item())
    ds_b = r.screen_grads().cpu().numpy().astype(np.float64)
    rms = np.sqrt(np.mean(ds_a.reshape(-1, 10) ** 2, axis=0))
    assert np.all(np.abs(ds_b - ds_a).reshape(-1, 10) <= 1e-4 * (np.abs(ds_a).reshape(-1, 10) + rms))
    # the two-launch form: the loss formed inside the render backward (gsr_render_bwd_l1)
    r.dinst.fill_(-7)
    loss_c = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = torch.empty((gsr.render_bwd_l1_workspace(V, raster) + 255) // 256 * 64, dtype=torch.int32, device="cuda")
    gsr.render_bwd_l1(r.splats, r.inst_gid, r.inst_emit, r.tile_ranges, ct, V, raster, r.rgb, r.depth, r.T_final,
                      r.last, trgb, tdep, 0.2, loss_c, r.dinst, ws, tile_order=r.tile_order)
    torch.cuda.synchronize()
    assert abs(loss_a.item() - loss_c.item()) <= 1e-12 * abs(loss_a.item())
    ds_c = r.screen_grads().cpu().numpy().astype(np.float64)
    assert np.all(np.abs(ds_c - ds_a).reshape(-1, 10) <= 1e-4 * (np.abs(ds_a).reshape(-1, 10) + rms))
    # the timed step's form: the sliced forward, then the L1 backward with the long tiles in its depth
    # slices (the forward's workspace handed over)
    r.dinst.fill_(-7)
    gsr.render_fwd(r.splats, r.inst_gid, r.tile_ranges, ct, V, raster, r.rgb, r.depth, r.T_final, r.last,
                   tile_order=r.tile_order, ws=r.fwd_ws, capacity=r.capacity)
    loss_d = torch.zeros(1, dtype=torch.float64, device="cuda")
    gsr.render_bwd_l1(r.splats, r.inst_gid, r.inst_emit, r.tile_ranges, ct, V, raster, r.rgb, r.depth, r.T_final,
                      r.last, trgb, tdep, 0.2, loss_d, r.dinst, ws, tile_order=r.tile_order, fwd_ws=r.fwd_ws,
                      capacity=r.capacity)
    torch.cuda.synchronize()
    assert torch.equal(r.rgb, ref["rgb"]) and torch.equal(r.T_final, ref["T"]) and torch.equal(r.last, ref["last"])
    assert abs(loss_a.item() - loss_d.item()) <= 1e-12 * abs(loss_a.item())
    ds_d = r.screen_grads().cpu().numpy().astype(np.float64)
    assert np.all(np.abs(ds_d - ds_a).reshape(-1, 10) <= 1e-4 * (np.abs(ds_a).reshape(-1, 10) + rms))


@pytest.mark.parametrize("n", [0, 15, 4099])
def test_step_prep_matches_torch(n):
    """gsr_step_prep against the torch ops it stands for: the camera gather (index_select), the
    int32 copy of the view indices, the cleared loss, the advanced step and the cleared row mask
    (lengths with and without a partial 16-byte group)."""
    import paper_2604_12942_amd as gsr
    rng = np.random.default_rng(n)
    S, V = 7, 5
    pool = torch.from_numpy(rng.integers(0, 256, S * 96, dtype=np.uint8)).cuda()
    idx = torch.tensor([3, 0, 6, 3, 1], dtype=torch.int64, device="cuda")
    cams = torch.zeros(V * 96, dtype=torch.uint8, device="cuda")
    idx32 = torch.full((V,), -1, dtype=torch.int32, device="cuda")
    loss = torch.full((1,), 5.0, dtype=torch.float64, device="cuda")
    step = torch.full((1,), 41, dtype=torch.int32, device="cuda")
    mask = torch.ones(n, dtype=torch.uint8, device="cuda")
    gsr.step_prep(pool, idx, cams, idx32, loss=loss, step=step, row_mask=mask if n else None)
    ref = torch.index_select(pool.view(S, 96), 0, idx).reshape(-1)
    assert torch.equal(cams, ref)
    assert idx32.tolist() == idx.tolist()
    assert loss.item() == 0.0 and step.item() == 42
    assert int(mask.sum()) == 0
    # only the camera gather: the optional outputs are left as they were
    loss.fill_(3.0)
    gsr.step_prep(pool, idx.flip(0).contiguous(), cams)
    assert torch.equal(cams, torch.index_select(pool.view(S, 96), 0, idx.flip(0)).reshape(-1))
    assert loss.item() == 3.0 and step.item() == 42


def test_pair_sums_are_ordered_record_sums():
    """gsr_pair_grads: the screen-space gradient of a (view, Gaussian) pair is the sum of its
    instance records.  Pairs of at most 32 records (the kernel sums every pair of up to 64 in
    emission order) equal a sequential float32 sum bit for bit; larger pairs (a few Gaussians
    blown up to cover most tiles) are checked to float rounding."""
    import paper_2604_12942_amd as gsr
    g, cams, _, _ = _three_views(5)
    g = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in g.items()}
    g["log_scales"][:, :16] += 2.5
    V = len(cams)
    H, W = cams[0]["height"], cams[0]["width"]
    P = gsr.gaussians_to_device(g)
    ct = gsr.camera_tensor(cams)
    n = P["means"].shape[1]
    r = gsr.Rasterizer(n, V, gsr.Raster(W, H))
    r.forward(P, g["sh_degree"], ct)
    rng = np.random.default_rng(2)
    gC = torch.from_numpy(rng.standard_normal((V, 3, H, W)).astype(np.float32)).cuda()
    gD = torch.from_numpy(rng.standard_normal((V, H, W)).astype(np.float32)).cuda()
    r.render_backward(ct, gC, gD)
    ds = r.screen_grads().cpu().numpy().reshape(-1, 10)
    npairs = int(r.n_pairs.item())
    first = r.pair_first[:npairs].cpu().numpy().astype(np.int64)
    gid = r.pair_gid[:npairs].cpu().numpy().astype(np.int64)
    ntiles = r.tile_info.view(4, -1)[0].cpu().numpy().astype(np.int64)
    cnt = np.append(first[1:] - first[:-1], ntiles[gid[-1]])
    total = int(first[-1] + cnt[-1])
    rec = r.dinst[:total * 10].cpu().numpy().reshape(-1, 10)
    small = cnt <= 32
    assert small.any() and (~small).any(), (cnt.min(), cnt.max())
    acc = np.zeros((npairs, 10), np.float32)
    for j in range(32):
        m = small & (cnt > j)
        acc[m] += rec[first[m] + j]
    assert np.array_equal(ds[gid[small]], acc[small])
    for q in np.flatnonzero(~small):
        part = rec[first[q]:first[q] + cnt[q]].astype(np.float64)
        assert np.all(np.abs(ds[gid[q]] - part.sum(0)) <= 1e-5 * (np.abs(part).sum(0) + 1e-30)), q
