"""Shared helpers of the GPU parity tests: run the HIP path on seeded inputs, compare with the
oracle under the stated tolerances."""
import numpy as np
import torch

import paper_2604_12942_amd as gsr

# Images and projected values: |g - o| <= 1e-5 max(|o|, 1e-2 max|o|)   (1e-5 relative)
IMG_RTOL = 1e-5
# Gradients: |g - o| <= 1e-3 (|o| + rms(o))                              (1e-3 relative)
GRAD_RTOL = 1e-3
# Decision-margin threshold of a knife-edge pixel
KNIFE = 1e-5


def img_close(g, o, rtol=IMG_RTOL, mask=None):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    tol = rtol * np.maximum(np.abs(o), 1e-2 * np.abs(o).max() if o.size else 0.0)
    bad = np.abs(g - o) > tol
    if mask is not None:
        bad &= mask
    return bad


def grad_close(g, o, rtol=GRAD_RTOL, mask=None):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    sel = o if mask is None else o[..., mask]
    rms = np.sqrt(np.mean(sel ** 2)) if sel.size else 0.0
    bad = np.abs(g - o) > rtol * (np.abs(o) + rms)
    if mask is not None:
        bad &= mask
    return bad


def run_forward(g, cams, tile=(16, 16), capacity=None, mode="recompute", sliced=True):
    """HIP forward of all cams (same size).  Returns dict of numpy outputs and the state.
    sliced=False: every tile composited whole."""
    W, H = cams[0]["width"], cams[0]["height"]
    raster = gsr.Raster(W, H, *tile)
    P = gsr.gaussians_to_device(g)
    n = P["means"].shape[1]
    ct = gsr.camera_tensor(cams)
    rast = gsr.Rasterizer(n, len(cams), raster, capacity=capacity, mode=mode)
    rgb, depth, Tf = rast.forward(P, g["sh_degree"], ct, sliced=sliced)
    torch.cuda.synchronize()
    out = dict(rgb=rgb.cpu().numpy().astype(np.float64), depth=depth.cpu().numpy().astype(np.float64),
               T=Tf.cpu().numpy().astype(np.float64), last=rast.last.cpu().numpy(), M=rast.instances())
    return out, rast, P, ct


def splat_fields(rast):
    """Decode the 48-byte splat records: u, v (float64), l11, l21, l22, opacity, depth, r, g, b."""
    raw = rast.splats.cpu().numpy().view(np.uint8).reshape(-1, 48)
    uv = raw[:, :16].copy().view(np.float64).reshape(-1, 2)
    # records of pairs no tile uses are never written: their bytes may be signalling NaNs
    with np.errstate(invalid="ignore"):
        f = raw[:, 16:].copy().view(np.float32).reshape(-1, 8).astype(np.float64)
    return dict(u=uv[:, 0], v=uv[:, 1], l11=f[:, 0], l21=f[:, 1], l22=f[:, 2], opacity=f[:, 3], depth=f[:, 4],
                r=f[:, 5], g=f[:, 6], b=f[:, 7])


def tile_info(rast):
    ti = rast.tile_info.cpu().numpy().view(np.uint32).reshape(4, -1)
    return dict(n_tiles=ti[0], zbits=ti[1], tx0=ti[2] & 0xFFFF, ty0=ti[2] >> 16, tx1=ti[3] & 0xFFFF, ty1=ti[3] >> 16)


def expected_instances(ti, n, V, raster, with_emission=False):
    """Reference order by numpy.lexsort on (view-tile, depth bits, pair index).  With
    with_emission, also each sorted instance's emission index (pairs in (depth bits, index)
    order, a pair's tiles row-major and consecutive) and each visible pair's first index."""
    keys, zb, gids, local = [], [], [], []
    vis = np.nonzero(ti["n_tiles"] > 0)[0]
    for gid in vis:
        v = gid // n
        j = 0
        for ty in range(ti["ty0"][gid], ti["ty1"][gid] + 1):
            for tx in range(ti["tx0"][gid], ti["tx1"][gid] + 1):
                keys.append(v * raster.tiles + ty * raster.ntx + tx)
                zb.append(ti["zbits"][gid])
                gids.append(gid)
                local.append(j)
                j += 1
    keys = np.asarray(keys, np.int64)
    zb = np.asarray(zb, np.int64)
    gids = np.asarray(gids, np.int64)
    local = np.asarray(local, np.int64)
    order = np.lexsort((gids, zb, keys))
    if not with_emission:
        return keys[order], gids[order]
    porder = vis[np.lexsort((vis, ti["zbits"][vis].astype(np.int64)))]
    cnt = ti["n_tiles"][porder].astype(np.int64)
    first = dict(zip(porder.tolist(), (np.cumsum(cnt) - cnt).tolist()))
    emit = np.array([first[g] for g in gids.tolist()], np.int64) + local
    return keys[order], gids[order], emit[order], first


def long_tile_scene(seed=11, W=64, H=64, f=60.0):
    """A vanishing-point pile-up on a 64x64 image: 48,000 small, faint Gaussians at depths 2-8 m
    crowd the four central 16x16 tiles (lists of about 11,000 instances, so the forward cuts them
    into depth slices of 1024), and 600 nearly opaque ones at 4.5-5.5 m, past the 4,000th list
    position, on which a few hundred central pixels terminate."""
    import synth
    faint = synth.random_gaussians(seed, 48_000, 1, xy_half=1.0, z_range=(2.0, 8.0), log_scale_mean=-2.3,
                                   log_scale_std=0.4)
    faint["opacity_logits"] = (faint["opacity_logits"] - 5.0).astype(np.float32)
    solid = synth.random_gaussians(seed + 1, 600, 1, xy_half=0.6, z_range=(4.5, 5.5), log_scale_mean=-2.8,
                                   log_scale_std=0.3)
    solid["opacity_logits"] = (solid["opacity_logits"] + 3.0).astype(np.float32)
    g = {k: np.concatenate([faint[k], solid[k]], axis=-1) if isinstance(faint[k], np.ndarray) else faint[k]
         for k in faint}
    cam = synth.make_camera(np.eye(3), np.zeros(3), f, f, W / 2.0, H / 2.0, W, H)
    return g, cam


def random_scene(seed, n, W, H, f, sh_degree=0, z_range=(1.5, 6.0), log_scale_mean=-2.5, xy_half=1.5, logit_shift=0.0):
    import synth
    g = synth.random_gaussians(seed, n, sh_degree, xy_half=xy_half, z_range=z_range,
                               log_scale_mean=log_scale_mean, log_scale_std=0.5)
    g["opacity_logits"] = (g["opacity_logits"] + logit_shift).astype(np.float32)
    cam = synth.make_camera(np.eye(3), np.zeros(3), f, f, W / 2.0, H / 2.0, W, H)
    return g, cam
