"""GPU parity of the point network (matrix-core forward, persistent backward) against the FP64
oracle with the same BF16 rounding points.

The oracle is fed the GPU's own float32 network inputs (the rows (p - mu) / 0.5 from the GPU's
voxel means, the 12 features from its eigenvalues and frames), so what is compared is the
network alone.  Every output and weight-gradient element is held at the gradient gate
|g - o| <= 1e-3 (|o| + rms(o)).  An element outside it is accepted only if it is a BF16 knife
edge: one that moves by more than a tenth of that tolerance when every value at a BF16 rounding
point is jittered by up to the float32 bound of its own evaluation (pointnet_oracle.knife_spread,
16 seeded realisations).  The number of such elements is reported."""
import numpy as np
import pytest
import torch

from oracle import init_oracle as io
from oracle import pointnet_oracle as pn
from test_gpu_init import _room_points

pytestmark = pytest.mark.gpu

ORDER = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4", "W5", "b5")
RTOL = 1e-3
KNIFE_FRAC = 0.1  # of the tolerance


def _gpu_inputs(pts, o, vox, nv):
    """The network inputs exactly as the GPU forms them, in float32."""
    mu = vox["mu"][:, :nv].cpu().numpy().T  # float32 [nv, 3]
    P32 = np.asarray(pts, np.float32)
    X = np.zeros((nv, pn.ROWS, 3), np.float32)
    for v in range(nv):
        ids = np.asarray(o["ids"][v])
        rows = ids[np.arange(pn.ROWS) % len(ids)]
        X[v] = (P32[rows] - mu[v]) / np.float32(0.5)
    lam = vox["evals"][:, :nv].cpu().numpy().T.astype(np.float32)
    R = vox["R"][:, :nv].cpu().numpy().T.reshape(nv, 3, 3)
    logl = np.log(np.maximum(lam, np.float32(0.005) * np.float32(0.005)) / np.float32(0.25)).astype(np.float32)
    F = np.concatenate([logl, R[:, :, 2], R[:, :, 1], R[:, :, 0]], axis=1)
    return X.astype(np.float64), F.astype(np.float64)


def _setup(n=24000, seed=3):
    import paper_2604_12942_amd as gsr
    pts, col, rng_, seg = _room_points(n, seed=seed)
    t = torch.from_numpy(np.ascontiguousarray(pts.T)).cuda()
    vox = gsr.voxel_pca(t, 17)
    o = io.voxel_pca(pts, 17)
    nv = len(o["n"])
    assert int(vox["n_voxels"].item()) == nv
    X, F = _gpu_inputs(pts, o, vox, nv)
    rng = np.random.default_rng(seed)
    W = pn.init_weights(seed)
    for k in ("b1", "b2", "b3", "b4", "b5"):
        W[k] = (rng.standard_normal(W[k].shape) * 0.1).astype(np.float32)
    flat = np.concatenate([W[k].ravel() for k in ORDER]).astype(np.float32)
    assert flat.size == gsr.pointnet_weight_count()
    return gsr, t, vox, o, X, F, W, torch.from_numpy(flat).cuda(), rng


def _gate(got, exp, spread_fn, axis=None):
    """Elements outside the 1e-3 gate; each must be a knife edge (the spread is computed only
    when there is one).  Returns (outside, outside and not a knife edge, total)."""
    rms = np.sqrt(np.mean(exp ** 2, axis=axis, keepdims=axis is not None)) + 1e-30
    tol = RTOL * (np.abs(exp) + rms)
    over = np.abs(got - exp) > tol
    if not over.any():
        return 0, 0, exp.size
    knife = spread_fn() > KNIFE_FRAC * tol
    return int(over.sum()), int((over & ~knife).sum()), exp.size


def test_pointnet_forward_matches_oracle():
    gsr, t, vox, o, X, F, W, wt, rng = _setup()
    nv = len(o["n"])
    y = gsr.pointnet_forward(t, vox, wt)
    torch.cuda.synchronize()
    got = y[:, :nv].cpu().numpy().T.astype(np.float64)
    exp = pn.forward(W, X, F)
    over, bad, total = _gate(got, exp, lambda: pn.knife_spread(W, X, F, realisations=16, seed=1)[0], axis=0)
    print("point network forward: %d of %d outputs outside 1e-3, all BF16 knife edges" % (over, total))
    assert bad == 0, (over, bad)
    assert over <= 1e-3 * total, over


def test_pointnet_backward_matches_oracle():
    gsr, t, vox, o, X, F, W, wt, rng = _setup(seed=4)
    nv = len(o["n"])
    n = t.shape[1]
    A = rng.standard_normal((nv, 3, 3)) * 0.05
    cov = A @ np.transpose(A, (0, 2, 1)) + np.eye(3) * 1e-3
    ot = rng.uniform(0.05, 0.95, nv)
    sel = rng.random(nv) < 0.8
    cov6 = np.zeros((6, n), np.float32)
    cov6[:, :nv] = np.stack([cov[:, 0, 0], cov[:, 0, 1], cov[:, 0, 2], cov[:, 1, 1], cov[:, 1, 2], cov[:, 2, 2]])
    o_t = np.zeros(n, np.float32)
    o_t[:nv] = ot
    mask = np.zeros(n, np.uint8)
    mask[:nv] = sel
    grad = torch.zeros(gsr.pointnet_weight_count(), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gsr.pointnet_backward(t, vox, wt, torch.from_numpy(cov6).cuda(), torch.from_numpy(o_t).cuda(),
                          torch.from_numpy(mask).cuda(), 1.0 / sel.sum(), grad, loss, blocks=64)
    torch.cuda.synchronize()
    cov32 = cov[sel].astype(np.float32).astype(np.float64)
    ot32 = ot[sel].astype(np.float32).astype(np.float64)
    y, keep = pn.forward(W, X[sel], F[sel], keep=True)
    L, dy = pn.loss(y, cov32, ot32)
    G = pn.backward(W, keep, dy, round_grads=True)
    got = grad.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - L) <= 1e-3 * abs(L)
    spread = {}

    def spread_of(k):
        if not spread:
            spread.update(pn.knife_spread(W, X[sel], F[sel], realisations=16, seed=2, cov_t=cov32, o_t=ot32)[1])
        return spread[k]

    off, stats, n_over, n_total = 0, {}, 0, 0
    for k in ORDER:
        m = G[k].size
        over, bad, total = _gate(got[off:off + m].reshape(G[k].shape), G[k], lambda k=k: spread_of(k))
        stats[k] = (over, bad, total)
        n_over += over
        n_total += total
        off += m
    print("point network backward: %d of %d weight-gradient elements outside 1e-3, all BF16 knife edges"
          % (n_over, n_total), stats)
    assert all(b == 0 for _, b, _ in stats.values()), stats
    assert n_over <= 1e-3 * n_total, stats


def _inputs_from_gpu_arrays(pts, vox, ids):
    """Network inputs of the voxels ids, in float32 as the GPU forms them, from the GPU's own voxel
    arrays (start, count, point order, means, eigenvalues, frames)."""
    n = pts.shape[0]
    start = vox["start"][:n].cpu().numpy().astype(np.int64)
    count = vox["count"][:n].cpu().numpy().astype(np.int64)
    order = vox["point_order"][:n].cpu().numpy().astype(np.int64)
    mu = vox["mu"].view(3, -1)[:, :n].cpu().numpy().T[ids]
    m = np.minimum(count[ids], pn.ROWS)
    rows = order[start[ids][:, None] + np.arange(pn.ROWS)[None, :] % m[:, None]]
    X = (np.asarray(pts, np.float32)[rows] - mu[:, None, :]) / np.float32(0.5)
    lam = vox["evals"].view(3, -1)[:, :n].cpu().numpy().T[ids].astype(np.float32)
    R = vox["R"].view(9, -1)[:, :n].cpu().numpy().T[ids].reshape(-1, 3, 3)
    logl = np.log(np.maximum(lam, np.float32(0.005) * np.float32(0.005)) / np.float32(0.25)).astype(np.float32)
    F = np.concatenate([logl, R[:, :, 2], R[:, :, 1], R[:, :, 0]], axis=1)
    return X.astype(np.float64), F.astype(np.float64)


def test_pointnet_forward_full_batch_sampled():
    """The timed batch (200k voxels of 32 points, 6.4M points) in the timed launch: the outputs of
    every voxel of the first and last three waves' ranges (whole and partial groups of 32, both
    staging halves) and of 2,048 random voxels against the oracle, under the same gate."""
    import synth
    import paper_2604_12942_amd as gsr
    pts, _, _, _ = synth.voxel_batch(0)
    t = torch.from_numpy(np.ascontiguousarray(pts.T)).cuda()
    vox = gsr.voxel_pca(t, 1)
    nv = int(vox["n_voxels"].item())
    assert nv == 200_000
    rng = np.random.default_rng(7)
    W = pn.init_weights(7)
    for k in ("b1", "b2", "b3", "b4", "b5"):
        W[k] = (rng.standard_normal(W[k].shape) * 0.1).astype(np.float32)
    flat = np.concatenate([W[k].ravel() for k in ORDER]).astype(np.float32)
    y = gsr.pointnet_forward(t, vox, torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    # the launch's wave ranges: persistent grid of min(ceil(ceil(n / 32) / 4), 3 CUs) workgroups
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n = pts.shape[0]
    nwaves = 4 * min(-(-(-(-n // 32)) // 4), 3 * cus)
    edge = [np.arange(g * nv // nwaves, (g + 1) * nv // nwaves) for g in (0, 1, 2, nwaves - 3, nwaves - 2, nwaves - 1)]
    ids = np.unique(np.concatenate(edge + [rng.choice(nv, 2048, replace=False)]))
    X, F = _inputs_from_gpu_arrays(pts, vox, ids)
    got = y.view(8, -1)[:, ids].cpu().numpy().T.astype(np.float64)
    exp = pn.forward(W, X, F)
    over, bad, total = _gate(got, exp, lambda: pn.knife_spread(W, X, F, realisations=16, seed=3)[0], axis=0)
    print("point network forward, %d sampled voxels of 200k: %d of %d outputs outside 1e-3, all BF16 knife edges"
          % (len(ids), over, total))
    assert bad == 0, (over, bad)
    assert over <= 1e-3 * total, over
