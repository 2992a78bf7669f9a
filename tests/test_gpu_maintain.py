"""GPU parity of the map maintenance (Sec. III-C) against the oracle: the pruning selection and
the proximity filter are integer results (bit-exact); row gathers are exact copies."""
import numpy as np
import pytest
import torch

import synth
from oracle import maintain_oracle as mo

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,ratio", [(300_000, 0.0), (300_000, 0.02), (300_000, 0.3), (4097, 1.0), (1, 1.0)])
def test_prune_select_bit_exact(n, ratio):
    import paper_2604_12942_amd as gsr
    rng = np.random.default_rng(n % 1000 + int(ratio * 100))
    lg = rng.normal(-1.0, 2.0, n).astype(np.float32)
    lg[rng.integers(0, n, n // 50)] = np.float32(-3.25)  # many equal logits across the cut
    seg = rng.integers(0, 8, n).astype(np.int32)
    thr = np.float32(-2.0)
    keep, n_keep = gsr.prune_select(torch.from_numpy(lg).cuda(), float(thr), ratio, torch.from_numpy(seg).cuda(), 3)
    torch.cuda.synchronize()
    k = int(n_keep.item())
    got = keep[:k].cpu().numpy().view(np.uint32).astype(np.int64)
    exp, _ = mo.prune_select(lg, thr, ratio, seg, 3)
    assert k == exp.size
    assert np.array_equal(got, exp)
    # without segment ids every candidate is eligible
    keep, n_keep = gsr.prune_select(torch.from_numpy(lg).cuda(), float(thr), ratio)
    torch.cuda.synchronize()
    exp, _ = mo.prune_select(lg, thr, ratio)
    assert np.array_equal(keep[:int(n_keep.item())].cpu().numpy().view(np.uint32).astype(np.int64), exp)


def test_prune_empty():
    import paper_2604_12942_amd as gsr
    keep, n_keep = gsr.prune_select(torch.zeros(0, device="cuda"), -1.0, 0.5)
    torch.cuda.synchronize()
    assert int(n_keep.item()) == 0


def test_gather_rows_compact_and_append():
    import paper_2604_12942_amd as gsr
    rng = np.random.default_rng(1)
    n, m = 70_001, 3_333
    A = rng.standard_normal((5, n)).astype(np.float32)
    S = rng.integers(0, 9, n).astype(np.int32)
    idx = np.sort(rng.choice(n, 40_000, replace=False)).astype(np.int32)
    dA = torch.empty(5, idx.size, device="cuda")
    dS = torch.empty(idx.size, dtype=torch.int32, device="cuda")
    gsr.gather_rows([(torch.from_numpy(A).cuda(), dA), (torch.from_numpy(S).cuda(), dS)], n,
                    torch.from_numpy(idx).cuda(), idx.size, idx.size)
    torch.cuda.synchronize()
    assert np.array_equal(dA.cpu().numpy(), mo.gather_rows(A, idx))
    assert np.array_equal(dS.cpu().numpy(), mo.gather_rows(S, idx))
    # append: old rows by identity, then the new rows picked by an index list
    B = rng.standard_normal((5, m)).astype(np.float32)
    bi = np.array([0, 5, 17, m - 1], np.int32)
    out = torch.empty(5, n + bi.size, device="cuda")
    gsr.gather_rows([(torch.from_numpy(A).cuda(), out)], n, None, n, n + bi.size, 0)
    gsr.gather_rows([(torch.from_numpy(B).cuda(), out)], m, torch.from_numpy(bi).cuda(), bi.size, n + bi.size, n)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.concatenate([A, B[:, bi]], axis=1))


def _points(seed, n_map, n_new, d):
    rng = np.random.default_rng(seed)
    A = np.concatenate([rng.uniform(-20, 20, (3, n_map // 2)),
                        rng.normal(0, 0.5, (3, n_map - n_map // 2)) + np.array([[3.0], [-2.0], [1.0]])], axis=1)
    pick = rng.integers(0, A.shape[1], n_new // 2)
    near = A[:, pick] + rng.normal(0, 0.6 * d, (3, pick.size))  # many near the decision
    far = rng.uniform(-20, 20, (3, n_new - pick.size))
    return A.astype(np.float32), np.concatenate([near, far], axis=1).astype(np.float32)


@pytest.mark.parametrize("d", [0.05, 0.3])
def test_proximity_filter_bit_exact(d):
    import paper_2604_12942_amd as gsr
    A, B = _points(int(d * 100), 30_000, 10_000, d)
    keep, idx, n_keep = gsr.proximity_filter(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), d)
    torch.cuda.synchronize()
    red = mo.redundant(A, B, d)
    got = keep[:B.shape[1]].cpu().numpy().astype(bool)
    assert np.array_equal(got, ~red), int((got != ~red).sum())
    k = int(n_keep.item())
    assert np.array_equal(idx[:k].cpu().numpy(), np.nonzero(~red)[0])
    assert 0 < red.sum() < B.shape[1]


def test_proximity_filter_large_map_sampled():
    """A 1.5M-mean map (the loop corridor) against 60k new means: every sampled decision matches
    the brute-force oracle."""
    import paper_2604_12942_amd as gsr
    c = synth.config3(n_points=1_500_000)
    A = np.ascontiguousarray(c["gaussians"]["means"], np.float32)
    rng = np.random.default_rng(7)
    d = 0.05
    pick = rng.integers(0, A.shape[1], 40_000)
    B = np.concatenate([A[:, pick] + rng.normal(0, 0.6 * d, (3, pick.size)),
                        A[:, rng.integers(0, A.shape[1], 20_000)] + rng.normal(0, 0.5, (3, 20_000))],
                       axis=1).astype(np.float32)
    keep, idx, n_keep = gsr.proximity_filter(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), d)
    torch.cuda.synchronize()
    got = keep[:B.shape[1]].cpu().numpy().astype(bool)
    s = rng.choice(B.shape[1], 150, replace=False)
    red = mo.redundant(A, B[:, s], d)
    assert np.array_equal(got[s], ~red)
    assert int(n_keep.item()) == int(got.sum())


def test_proximity_edge_cases():
    import paper_2604_12942_amd as gsr
    a = torch.zeros(3, 1, device="cuda")
    b = torch.tensor([[0.25, 0.2499], [0.0, 0.0], [0.0, 0.0]], device="cuda")
    keep, _, n_keep = gsr.proximity_filter(a, b, 0.25)
    torch.cuda.synchronize()
    assert keep.cpu().tolist() == [1, 0]  # exactly d_min apart is not redundant
    keep, idx, n_keep = gsr.proximity_filter(torch.zeros(3, 0, device="cuda"), b, 0.25)
    torch.cuda.synchronize()
    assert keep.cpu().tolist() == [1, 1] and int(n_keep.item()) == 2
    keep, idx, n_keep = gsr.proximity_filter(a, torch.zeros(3, 0, device="cuda"), 0.25)
    torch.cuda.synchronize()
    assert int(n_keep.item()) == 0


def test_optimizer_prune_and_insert():
    """Pruning and insertion inside the optimiser: parameters, Adam moments and segment ids of
    the survivors are exactly the old rows; the optimiser keeps stepping, also from a recaptured
    graph."""
    import paper_2604_12942_amd as gsr
    from paper_2604_12942_amd.optimize import MapOptimizer
    c = synth.config4a()
    g = c["gaussians"]
    rng = np.random.default_rng(0)
    cams = [c["cameras"][0]] + [synth.make_camera(synth.small_rotation(rng, 8.0), rng.uniform(-0.2, 0.2, 3), 125.0,
                                                  125.0, 80.0, 60.0, 160, 120) for _ in range(2)]
    trgb = torch.from_numpy(rng.uniform(0, 1, (3, 3, 120, 160)).astype(np.float32)).cuda()
    tdep = torch.from_numpy(rng.uniform(2, 10, (3, 120, 160)).astype(np.float32)).cuda()
    n = g["means"].shape[1]
    seg = torch.from_numpy((np.arange(n) % 4).astype(np.int32)).cuda()
    P = gsr.gaussians_to_device(g)
    opt = MapOptimizer(P, g["sh_degree"], gsr.camera_tensor(cams), trgb, tdep, gsr.Raster(160, 120), 3,
                       segment_id=seg, min_segment=2)
    for s in range(3):
        opt.set_views([0, 1, 2])
        opt.step()
    torch.cuda.synchronize()
    old = {k: t.cpu().numpy().copy() for k, t in opt._row_arrays().items()}
    removed = opt.prune(min_opacity=0.3, max_ratio=0.1)
    torch.cuda.synchronize()
    keep, _ = mo.prune_select(old["opacity_logits"].reshape(-1), np.log(0.3 / 0.7), 0.1, old["segment_id"], 2)
    assert removed == n - keep.size and 0 < removed <= n // 10
    new = {k: t.cpu().numpy() for k, t in opt._row_arrays().items()}
    for k in old:
        assert np.array_equal(new[k], old[k][..., keep]), k
    # insert: half the new means duplicate existing ones
    m = 400
    src = rng.integers(0, opt.n, m)
    means = new["means"][:, src].copy()
    means[:, m // 2:] += rng.normal(0, 0.5, (3, m - m // 2)).astype(np.float32)
    add = {k: torch.from_numpy(np.ascontiguousarray(new[k][..., src])).cuda() for k in gsr.PARAM_NAMES}
    add["means"] = torch.from_numpy(means).cuda()
    n0 = opt.n
    added = opt.insert(add, torch.full((m,), 3, dtype=torch.int32, device="cuda"), d_min=0.05)
    torch.cuda.synchronize()
    red = mo.redundant(new["means"], means, 0.05)
    assert added == int((~red).sum()) and opt.n == n0 + added
    after = {k: t.cpu().numpy() for k, t in opt._row_arrays().items()}
    assert np.array_equal(after["means"][:, n0:], means[:, ~red])
    assert not after["m_means"][:, n0:].any()
    opt.set_views([2, 0, 1])
    l1 = float(opt.step().item())
    opt.capture()
    opt.set_views([1, 2, 0])
    l2 = float(opt.replay().item())
    torch.cuda.synchronize()
    assert np.isfinite(l1) and np.isfinite(l2)


@pytest.mark.parametrize("n,with_seg", [(300_000, True), (300_000, False), (4097, True), (1, True)])
def test_row_order_bit_exact(n, with_seg):
    import paper_2604_12942_amd as gsr
    rng = np.random.default_rng(n % 997)
    m = rng.uniform(-40, 60, (3, n)).astype(np.float32)
    m[:, rng.integers(0, n, n // 100)] = m[:, :1]  # repeated means: ties kept in row order
    seg = rng.integers(-2, 20, n).astype(np.int32) if with_seg else None
    order = gsr.row_order(torch.from_numpy(m).cuda(), torch.from_numpy(seg).cuda() if with_seg else None)
    torch.cuda.synchronize()
    got = order[:n].cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(got, mo.row_order(m, seg))


def test_row_order_flat_box():
    import paper_2604_12942_amd as gsr
    m = np.tile(np.array([[1.5], [-2.0], [3.0]], np.float32), (1, 1000))
    seg = np.repeat(np.arange(4, dtype=np.int32), 250)[::-1].copy()
    order = gsr.row_order(torch.from_numpy(m).cuda(), torch.from_numpy(seg).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(order.cpu().numpy().astype(np.int64), mo.row_order(m, seg))


def test_optimizer_reorder_keeps_the_step():
    """A step on the reordered map is the step on the original map, rows permuted: loss and
    parameters agree to float rounding (depth ties aside, which this scene has none of)."""
    import paper_2604_12942_amd as gsr
    from paper_2604_12942_amd.optimize import MapOptimizer
    c = synth.config4a()
    g = c["gaussians"]
    rng = np.random.default_rng(1)
    cams = [c["cameras"][0]] + [synth.make_camera(synth.small_rotation(rng, 8.0), rng.uniform(-0.2, 0.2, 3), 125.0,
                                                  125.0, 80.0, 60.0, 160, 120) for _ in range(2)]
    trgb = torch.from_numpy(rng.uniform(0, 1, (3, 3, 120, 160)).astype(np.float32)).cuda()
    tdep = torch.from_numpy(rng.uniform(2, 10, (3, 120, 160)).astype(np.float32)).cuda()
    n = g["means"].shape[1]
    segs = rng.integers(0, 4, n).astype(np.int32)

    def make():
        return MapOptimizer(gsr.gaussians_to_device(g), g["sh_degree"], gsr.camera_tensor(cams), trgb, tdep,
                            gsr.Raster(160, 120), 3, segment_id=torch.from_numpy(segs).cuda(), min_segment=2)
    a, b = make(), make()
    order = b.reorder().cpu().numpy().view(np.uint32).astype(np.int64)
    torch.cuda.synchronize()
    assert np.array_equal(b.segment_id.cpu().numpy(), segs[order])
    for s in range(3):
        a.set_views([0, 1, 2] if s % 2 == 0 else [2, 0, 1])
        b.set_views([0, 1, 2] if s % 2 == 0 else [2, 0, 1])
        la, lb = float(a.step().item()), float(b.step().item())
        assert abs(la - lb) <= 1e-5 * abs(la)
    torch.cuda.synchronize()
    for k in gsr.PARAM_NAMES:
        pa = a.P[k].cpu().numpy()[..., order]
        pb = b.P[k].cpu().numpy()
        assert np.allclose(pa, pb, rtol=2e-6, atol=1e-6), k
