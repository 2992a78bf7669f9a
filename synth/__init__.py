"""Seeded synthetic inputs shared by the HIP path and the FP64 oracle.

This module only *draws* inputs: Gaussian parameters, cameras, LiDAR-like
point clouds and ray-traced target images of analytic scenes.  It contains
none of the rasterizer's arithmetic (no projection, compositing, gradients
or optimizer), so both sides can consume it without sharing method code.

Conventions (inputs only):
  * Gaussian parameters are structure-of-arrays, component-major, float32:
      means (3, N), log_scales (3, N), quats (4, N) as raw (w, x, y, z),
      opacity_logits (N,), sh (3*K, N) with row k*3+ch for SH coefficient k
      and colour channel ch, K = (degree+1)^2.
  * A camera is a dict with a world->camera rotation R (3x3, row-major) and
    translation t (3,), so p_cam = R @ mu + t; the camera looks along +z,
    image x to the right, image y down; pinhole fx, fy, cx, cy; integer
    width, height; z_near; background colour bg (3,).
  * Target images are float32 (3, H, W) colour and (H, W) depth.
"""
from __future__ import annotations

import numpy as np

Y00_INV = 2.0 * np.sqrt(np.pi)  # colour -> DC coefficient for the stand-in init


def make_camera(R, t, fx, fy, cx, cy, width, height, z_near=0.2, bg=(0.0, 0.0, 0.0)):
    return dict(R=np.asarray(R, np.float32).reshape(3, 3), t=np.asarray(t, np.float32).reshape(3),
                fx=float(fx), fy=float(fy), cx=float(cx), cy=float(cy),
                width=int(width), height=int(height), z_near=float(z_near),
                bg=np.asarray(bg, np.float32).reshape(3))


def look_camera(center, yaw, pitch, fx, fy, cx, cy, width, height, z_near=0.2):
    """Camera at `center` (world, z up) looking along yaw (about +z) and pitch (negative = down)."""
    f = np.array([np.cos(yaw) * np.cos(pitch), np.sin(yaw) * np.cos(pitch), np.sin(pitch)])
    up = np.array([0.0, 0.0, 1.0])
    r = np.cross(f, up)
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ np.asarray(center, np.float64)
    return make_camera(R, t, fx, fy, cx, cy, width, height, z_near)


def _random_unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    return q / np.linalg.norm(q, axis=0, keepdims=True)


def random_gaussians(seed, n, sh_degree, xy_half=2.0, z_range=(2.0, 10.0),
                     log_scale_mean=-3.0, log_scale_std=0.5, sh_rest_std=0.3):
    """Uniform Gaussians in a box in front of an identity camera.

    Draw order from default_rng(seed): means x, y, z; log-scales; quaternions;
    opacity logits; SH DC; SH rest.
    """
    rng = np.random.default_rng(seed)
    K = (sh_degree + 1) ** 2
    mx = rng.uniform(-xy_half, xy_half, n)
    my = rng.uniform(-xy_half, xy_half, n)
    mz = rng.uniform(z_range[0], z_range[1], n)
    means = np.stack([mx, my, mz])
    log_scales = rng.normal(log_scale_mean, log_scale_std, (3, n))
    quats = _random_unit_quats(rng, n)
    opacity_logits = rng.standard_normal(n)
    sh = np.zeros((3 * K, n))
    sh[0:3] = rng.standard_normal((3, n))
    if K > 1:
        sh[3:] = rng.normal(0.0, sh_rest_std, (3 * (K - 1), n))
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    return dict(means=f32(means), log_scales=f32(log_scales), quats=f32(quats),
                opacity_logits=f32(opacity_logits), sh=f32(sh), sh_degree=sh_degree)


def config1(seed=0):
    """2,000 Gaussians, SH degree 0, one identity camera 128x96, fx=fy=100; uniform target."""
    g = random_gaussians(seed, 2000, 0)
    cam = make_camera(np.eye(3), np.zeros(3), 100.0, 100.0, 64.0, 48.0, 128, 96)
    rng = np.random.default_rng(seed + 1000)
    tgt = rng.uniform(0.0, 1.0, (3, 96, 128)).astype(np.float32)
    return dict(gaussians=g, cameras=[cam], target_rgb=[tgt], target_depth=[None], lambda_depth=0.0)


def small_rotation(rng, max_deg):
    axis = rng.standard_normal(3)
    axis /= np.linalg.norm(axis)
    ang = np.deg2rad(rng.uniform(0.0, max_deg))
    Kx = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(ang) * Kx + (1 - np.cos(ang)) * Kx @ Kx


def config4a(seed=3, n=5000, width=160, height=120, f=125.0):
    """5k Gaussians, SH degree 3, 160x120, a random pose within 10 degrees / 0.2 m of identity."""
    g = random_gaussians(seed, n, 3)
    rng = np.random.default_rng(seed + 1000)
    R = small_rotation(rng, 10.0)
    t = rng.uniform(-0.2, 0.2, 3)
    cam = make_camera(R, t, f, f, width / 2.0, height / 2.0, width, height)
    tgt = rng.uniform(0.0, 1.0, (3, height, width)).astype(np.float32)
    tgt_d = rng.uniform(2.0, 10.0, (height, width)).astype(np.float32)
    return dict(gaussians=g, cameras=[cam], target_rgb=[tgt], target_depth=[tgt_d], lambda_depth=0.2)


# ---------------------------------------------------------------------------------------------
# Analytic LiDAR scenes: ground plane, axis-aligned vertical walls, yawed boxes on the ground.
# ---------------------------------------------------------------------------------------------

class Scene:
    """Analytic scene made of a ground plane (z=0), vertical wall rectangles and yawed boxes.

    walls: list of (axis, coord, lo, hi, height, normal_sign) meaning the plane
    {axis == coord} restricted to the other horizontal coordinate in [lo, hi]
    and z in [0, height]; normal_sign picks the side the wall faces.
    boxes: array (B, 7) of centre x, y, half-sizes a, b, c (height 2c, resting on z=0), yaw, id.
    """

    def __init__(self, walls, boxes, ground_extent, seed):
        self.walls = walls
        self.boxes = np.asarray(boxes, np.float64).reshape(-1, 7)
        self.ground_extent = ground_extent  # (xmin, xmax, ymin, ymax)
        rng = np.random.default_rng(seed + 777)
        n_surf = 1 + len(walls) + len(self.boxes)
        self.base_colour = rng.uniform(0.25, 0.9, (n_surf, 3))
        self.noise_seed = seed

    # -- procedural albedo (a deterministic function of position and surface id) --------------
    def _value_noise(self, p, scale, salt):
        g = np.floor(p / scale).astype(np.int64)
        f = p / scale - g
        f = f * f * (3 - 2 * f)

        def h(ix, iy, iz):
            v = (ix * 73856093) ^ (iy * 19349663) ^ (iz * 83492791) ^ (salt * 2654435761 + self.noise_seed)
            v = (v ^ (v >> 13)) * 1274126177
            v = v ^ (v >> 16)
            return (v & 0xFFFF).astype(np.float64) / 65535.0

        out = 0.0
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    w = (f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1]) * \
                        (f[:, 2] if dz else 1 - f[:, 2])
                    out = out + w * h(g[:, 0] + dx, g[:, 1] + dy, g[:, 2] + dz)
        return out

    def albedo(self, p, surf):
        chk = (np.floor(p[:, 0] / 0.5) + np.floor(p[:, 1] / 0.5) + np.floor(p[:, 2] / 0.5)) % 2
        n = 0.65 * self._value_noise(p, 1.3, 1) + 0.35 * self._value_noise(p, 0.31, 2)
        shade = (0.7 + 0.3 * chk) * (0.55 + 0.45 * n)
        return np.clip(self.base_colour[surf] * shade[:, None], 0.0, 1.0)

    # -- ray casting ---------------------------------------------------------------------------
    def cast(self, o, d, max_range=np.inf):
        """Rays o (3,) or (n,3) + t d (n,3, unit).  Returns t, surface id (-1 = miss), normal (n,3)."""
        n = d.shape[0]
        o = np.broadcast_to(o, (n, 3))
        best = np.full(n, np.inf)
        surf = np.full(n, -1, np.int64)
        nrm = np.zeros((n, 3))
        # ground
        with np.errstate(divide="ignore", invalid="ignore"):
            tg = -o[:, 2] / d[:, 2]
        hx = o[:, 0] + tg * d[:, 0]
        hy = o[:, 1] + tg * d[:, 1]
        xmin, xmax, ymin, ymax = self.ground_extent
        ok = (d[:, 2] < 0) & (tg > 1e-6) & (hx >= xmin) & (hx <= xmax) & (hy >= ymin) & (hy <= ymax)
        best = np.where(ok, tg, best)
        surf = np.where(ok, 0, surf)
        nrm[ok] = (0.0, 0.0, 1.0)
        # walls
        for wi, (axis, coord, lo, hi, height, sgn) in enumerate(self.walls):
            other = 1 - axis
            with np.errstate(divide="ignore", invalid="ignore"):
                tw = (coord - o[:, axis]) / d[:, axis]
            ho = o[:, other] + tw * d[:, other]
            hz = o[:, 2] + tw * d[:, 2]
            ok = (tw > 1e-6) & (tw < best) & (ho >= lo) & (ho <= hi) & (hz >= 0) & (hz <= height)
            best = np.where(ok, tw, best)
            surf = np.where(ok, 1 + wi, surf)
            wn = np.zeros(3)
            wn[axis] = sgn
            nrm[ok] = wn
        # boxes (slab test in the box frame)
        nb0 = 1 + len(self.walls)
        for bi, (bx, by, a, b, c, yaw, _) in enumerate(self.boxes):
            # bounding-sphere prefilter: only rays passing within the sphere, in front of the
            # current nearest hit, get the slab test
            rad = np.sqrt(a * a + b * b + c * c)
            vx, vy, vz = bx - o[:, 0], by - o[:, 1], c - o[:, 2]
            proj = vx * d[:, 0] + vy * d[:, 1] + vz * d[:, 2]
            perp2 = vx * vx + vy * vy + vz * vz - proj * proj
            cand = np.nonzero((perp2 < rad * rad) & (proj > -rad) & (proj - rad < best))[0]
            if cand.size == 0:
                continue
            cs, sn = np.cos(yaw), np.sin(yaw)
            oc, dcn = o[cand], d[cand]
            ox = oc[:, 0] - bx
            oy = oc[:, 1] - by
            lx = cs * ox + sn * oy
            ly = -sn * ox + cs * oy
            lz = oc[:, 2] - c
            dx = cs * dcn[:, 0] + sn * dcn[:, 1]
            dy = -sn * dcn[:, 0] + cs * dcn[:, 1]
            dz = dcn[:, 2]
            with np.errstate(divide="ignore", invalid="ignore"):
                t1x, t2x = (-a - lx) / dx, (a - lx) / dx
                t1y, t2y = (-b - ly) / dy, (b - ly) / dy
                t1z, t2z = (-c - lz) / dz, (c - lz) / dz
            tminx, tmaxx = np.minimum(t1x, t2x), np.maximum(t1x, t2x)
            tminy, tmaxy = np.minimum(t1y, t2y), np.maximum(t1y, t2y)
            tminz, tmaxz = np.minimum(t1z, t2z), np.maximum(t1z, t2z)
            tmin = np.maximum(np.maximum(tminx, tminy), tminz)
            tmax = np.minimum(np.minimum(tmaxx, tmaxy), tmaxz)
            ok = (tmax >= tmin) & (tmin > 1e-6) & (tmin < best[cand])
            if not ok.any():
                continue
            sel = np.nonzero(ok)[0]
            idx = cand[sel]
            best[idx] = tmin[sel]
            surf[idx] = nb0 + bi
            # face normal: the slab that produced tmin
            ax = np.where(tmin == tminx, 0, np.where(tmin == tminy, 1, 2))[sel]
            ln = np.zeros((sel.size, 3))
            ln[np.arange(sel.size), ax] = -np.sign(np.stack([dx, dy, dz], 1)[sel, ax])
            wnx = cs * ln[:, 0] - sn * ln[:, 1]
            wny = sn * ln[:, 0] + cs * ln[:, 1]
            nrm[idx] = np.stack([wnx, wny, ln[:, 2]], 1)
        miss = ~np.isfinite(best) | (best > max_range)
        surf[miss] = -1
        return best, surf, nrm

    def render_gt(self, cam, chunk=1 << 18):
        """Ray-traced ground-truth colour (3,H,W) and camera-frame depth (H,W) at pixel centres."""
        W, H = cam["width"], cam["height"]
        R = cam["R"].astype(np.float64)
        t = cam["t"].astype(np.float64)
        C = -R.T @ t
        jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
        xs = ((ii + 0.5) - cam["cx"]) / cam["fx"]
        ys = ((jj + 0.5) - cam["cy"]) / cam["fy"]
        dc = np.stack([xs.ravel(), ys.ravel(), np.ones(W * H)], 1)
        dw = dc @ R  # camera ray directions in world (R^T d)
        nrm = np.linalg.norm(dw, axis=1, keepdims=True)
        dw = dw / nrm
        rgb = np.zeros((W * H, 3))
        depth = np.zeros(W * H)
        for s in range(0, W * H, chunk):
            e = min(W * H, s + chunk)
            tt, sf, _ = self.cast(C, dw[s:e])
            hit = sf >= 0
            p = C + tt[hit, None] * dw[s:e][hit]
            col = np.zeros((e - s, 3))
            col[hit] = self.albedo(p, sf[hit])
            rgb[s:e] = col
            dd = np.zeros(e - s)
            dd[hit] = tt[hit] / nrm[s:e, 0][hit]  # ray length along unit dir -> camera z
            depth[s:e] = dd
        return (rgb.T.reshape(3, H, W).astype(np.float32), depth.reshape(H, W).astype(np.float32))

    def lidar(self, rng, sensor_xy, n_rays, sensor_height=1.8, max_range=60.0, noise=0.02,
              elev_deg=(-25.0, 15.0), n_beams=32, az_step_deg=0.2):
        """Random ring-scan rays (beam, azimuth and scan position drawn uniformly from the
        32-beam x 0.2-degree pattern at the given scan positions); returns hit points,
        surface ids, normals and the sensor-to-point range."""
        sensor_xy = np.asarray(sensor_xy, np.float64).reshape(-1, 2)
        elev = np.deg2rad(np.linspace(elev_deg[0], elev_deg[1], n_beams))
        n_az = int(round(360.0 / az_step_deg))
        si = rng.integers(0, len(sensor_xy), n_rays)
        bi = rng.integers(0, n_beams, n_rays)
        ai = rng.integers(0, n_az, n_rays)
        az = np.deg2rad(ai * az_step_deg)
        el = elev[bi]
        d = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], 1)
        o = np.concatenate([sensor_xy[si], np.full((n_rays, 1), sensor_height)], 1)
        pts, sfs, nms, rng_out, scan = [], [], [], [], []
        chunk = 1 << 17
        for s in range(0, n_rays, chunk):
            e = min(n_rays, s + chunk)
            tt, sf, nm = self.cast(o[s:e], d[s:e], max_range)
            hit = sf >= 0
            r = tt[hit] + rng.normal(0.0, noise, hit.sum())
            pts.append(o[s:e][hit] + r[:, None] * d[s:e][hit])
            sfs.append(sf[hit])
            nms.append(nm[hit])
            rng_out.append(r)
            scan.append(si[s:e][hit])
        return (np.concatenate(pts), np.concatenate(sfs), np.concatenate(nms), np.concatenate(rng_out),
                np.concatenate(scan))


def lidar_point_cov(points, origins, sigma_range=0.02, sigma_angle=np.deg2rad(0.1), sigma_pose=0.01):
    """World-frame covariance of LiDAR points, [n, 6] = (xx, xy, xz, yy, yz, zz): range noise along
    the beam, angular noise (times the range) across it, and an isotropic pose term."""
    d = np.asarray(points, np.float64) - np.asarray(origins, np.float64)
    r = np.linalg.norm(d, axis=1)
    b = d / r[:, None]
    along = sigma_range ** 2
    across = (r * sigma_angle) ** 2
    C = (along - across)[:, None, None] * b[:, :, None] * b[:, None, :] + \
        (across + sigma_pose ** 2)[:, None, None] * np.eye(3)[None]
    return np.stack([C[:, 0, 0], C[:, 0, 1], C[:, 0, 2], C[:, 1, 1], C[:, 1, 2], C[:, 2, 2]], 1).astype(np.float32)


def voxel_batch(seed, n_voxels=200_000, pts_per_voxel=32, voxel=0.5):
    """A batch of occupied 0.5 m voxels with pts_per_voxel LiDAR-like points each, for the
    initialisation path at scale: voxels on a lattice (x, y across 50 m, 20 layers in z), 60 % of
    them a noisy plane patch (2 cm noise), 20 % a noisy bar, 20 % scattered.  Points keep 2 cm from
    the voxel faces.  Returns points [n, 3], colours [n, 3], sensor origins [n, 3] (one per 10 m
    tile, 1.8 m up) and ranges [n]."""
    rng = np.random.default_rng(seed)
    side = int(np.ceil(np.sqrt(n_voxels / 20)))
    idx = np.arange(n_voxels)
    kx, ky, kz = idx % side - side // 2, (idx // side) % side - side // 2, idx // (side * side) - 10
    base = np.stack([kx, ky, kz], 1).astype(np.float64) * voxel
    m = pts_per_voxel
    kind = rng.random(n_voxels)
    u = rng.uniform(0.04, voxel - 0.04, (n_voxels, m, 3))
    # plane: a random tilt of the local xy plane through the voxel centre
    nrm = rng.standard_normal((n_voxels, 3))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    c = voxel / 2
    d = u - c
    plane = u - (np.einsum("vmk,vk->vm", d, nrm) - rng.normal(0, 0.02, (n_voxels, m)))[..., None] * nrm[:, None, :]
    axis = rng.standard_normal((n_voxels, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    tt = rng.uniform(-0.2, 0.2, (n_voxels, m, 1))
    bar = c + tt * axis[:, None, :] + rng.normal(0, 0.02, (n_voxels, m, 3))
    loc = np.where((kind < 0.6)[:, None, None], plane, np.where((kind < 0.8)[:, None, None], bar, u))
    loc = np.clip(loc, 0.02, voxel - 0.02)
    pts = (base[:, None, :] + loc).reshape(-1, 3)
    tile = np.floor(pts[:, :2] / 10.0) * 10.0 + 5.0
    org = np.c_[tile, np.full(len(pts), 1.8)]
    rngs = np.linalg.norm(pts - org, axis=1)
    col = rng.uniform(0.1, 0.9, (n_voxels, 3)).repeat(m, axis=0)
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    return f32(pts), f32(col), f32(org), f32(rngs)


def _boxes_uniform(rng, n, lo, hi, start_id):
    c = rng.uniform(lo, hi, (n, 2))
    size = rng.uniform(0.3, 2.0, (n, 3))
    yaw = rng.uniform(0.0, 2 * np.pi, n)
    return np.column_stack([c, size / 2.0, yaw, np.arange(start_id, start_id + n)])


def room_scene(seed=1):
    """40 x 40 m room: ground, four 4 m walls at x, y = +-20 m and 40 random boxes."""
    rng = np.random.default_rng(seed)
    walls = [(0, -20.0, -20.0, 20.0, 4.0, 1.0), (0, 20.0, -20.0, 20.0, 4.0, -1.0),
             (1, -20.0, -20.0, 20.0, 4.0, 1.0), (1, 20.0, -20.0, 20.0, 4.0, -1.0)]
    boxes = _boxes_uniform(rng, 40, -18.0, 18.0, 0)
    return Scene(walls, boxes, (-20.0, 20.0, -20.0, 20.0), seed)


def loop_point(s, half_x=30.0, half_y=20.0):
    """Point and heading at arc length s along the 60 x 40 m rectangular loop (perimeter 200 m)."""
    L = 2 * (2 * half_x + 2 * half_y)
    s = np.mod(s, L)
    legs = [(2 * half_x, (-half_x, -half_y), 0.0), (2 * half_y, (half_x, -half_y), np.pi / 2),
            (2 * half_x, (half_x, half_y), np.pi), (2 * half_y, (-half_x, half_y), -np.pi / 2)]
    for length, (x0, y0), yaw in legs:
        if s <= length:
            return np.array([x0 + s * np.cos(yaw), y0 + s * np.sin(yaw)]), yaw
        s -= length
    return np.array([-half_x, -half_y]), 0.0


def corridor_scene(seed=2):
    """200 m rectangular loop corridor (centre line 60 x 40 m, width 6 m, 4 m walls) with
    200 boxes in 10 wall-side clusters."""
    rng = np.random.default_rng(seed)
    ox, oy, ix, iy = 33.0, 23.0, 27.0, 17.0
    walls = [(0, -ox, -oy, oy, 4.0, 1.0), (0, ox, -oy, oy, 4.0, -1.0),
             (1, -oy, -ox, ox, 4.0, 1.0), (1, oy, -ox, ox, 4.0, -1.0),
             (0, -ix, -iy, iy, 4.0, -1.0), (0, ix, -iy, iy, 4.0, 1.0),
             (1, -iy, -ix, ix, 4.0, -1.0), (1, iy, -ix, ix, 4.0, 1.0)]
    boxes = []
    for k in range(10):
        p, yaw = loop_point(10.0 + 20.0 * k)
        side = 1.0 if k % 2 == 0 else -1.0
        nrm = np.array([-np.sin(yaw), np.cos(yaw)]) * side
        tang = np.array([np.cos(yaw), np.sin(yaw)])
        for j in range(20):
            off = rng.uniform(1.2, 2.4)
            along = rng.uniform(-3.0, 3.0)
            c = p + nrm * off + tang * along
            size = rng.uniform(0.3, 1.2, 3)
            boxes.append([c[0], c[1], size[0] / 2, size[1] / 2, size[2] / 2, rng.uniform(0, 2 * np.pi),
                          len(boxes)])
    return Scene(walls, np.array(boxes), (-ox, ox, -oy, oy), seed)


def lidar_gaussians(scene, rng, sensor_xy, n_points, sh_degree=3, sh_rest_std=0.05,
                    inplane_log_scale=np.log(0.1), inplane_std=0.2, normal_log_scale=np.log(0.02),
                    opacity=0.1, oversample=1.15):
    """Exactly n_points LiDAR returns turned into Gaussians by a stand-in for the voxel-PCA
    initialisation: a flat disc per point aligned with the analytic surface normal (in-plane
    log-scale ~ N(log 0.1 m, 0.2^2), normal log-scale log 2 cm), a random in-plane spin,
    constant opacity 0.1, SH DC from the surface colour and SH rest ~ N(0, 0.05^2)."""
    pts, sfs, nms, rngs, scan = scene.lidar(rng, sensor_xy, int(n_points * oversample))
    while pts.shape[0] < n_points:
        p2, s2, n2, r2, c2 = scene.lidar(rng, sensor_xy, int(n_points * 0.5))
        pts, sfs, nms, rngs, scan = (np.concatenate([pts, p2]), np.concatenate([sfs, s2]),
                                     np.concatenate([nms, n2]), np.concatenate([rngs, r2]),
                                     np.concatenate([scan, c2]))
    keep = np.sort(rng.choice(pts.shape[0], n_points, replace=False))
    pts, sfs, nms, rngs, scan = pts[keep], sfs[keep], nms[keep], rngs[keep], scan[keep]
    col = scene.albedo(pts, sfs)
    n = n_points
    # quaternion whose local z axis is the surface normal, with a random spin about it
    z = nms / np.linalg.norm(nms, axis=1, keepdims=True)
    helper = np.where(np.abs(z[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    x = np.cross(helper, z)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    spin = rng.uniform(0, 2 * np.pi, n)
    xs = np.cos(spin)[:, None] * x + np.sin(spin)[:, None] * y
    ys = np.cross(z, xs)
    Rm = np.stack([xs, ys, z], axis=2)  # columns = local axes
    quats = _rot_to_quat(Rm)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((3 * K, n))
    sh[0:3] = ((col - 0.5) * Y00_INV).T
    if K > 1:
        sh[3:] = rng.normal(0.0, sh_rest_std, (3 * (K - 1), n))
    ls = np.stack([rng.normal(inplane_log_scale, inplane_std, n), rng.normal(inplane_log_scale, inplane_std, n),
                   np.full(n, normal_log_scale)])
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    g = dict(means=f32(pts.T), log_scales=f32(ls), quats=f32(quats.T),
             opacity_logits=f32(np.full(n, np.log(opacity / (1 - opacity)))), sh=f32(sh), sh_degree=sh_degree)
    return g, dict(points=f32(pts), colors=f32(col), normals=f32(nms), ranges=f32(rngs), surface=sfs,
                   scan=scan)


def _rot_to_quat(Rm):
    """Rotation matrices (n,3,3) -> unit quaternions (n,4) as (w,x,y,z), w >= 0 (input synthesis)."""
    tr = Rm[:, 0, 0] + Rm[:, 1, 1] + Rm[:, 2, 2]
    q = np.zeros((Rm.shape[0], 4))
    m = [np.maximum(0.0, 1 + tr), np.maximum(0.0, 1 + Rm[:, 0, 0] - Rm[:, 1, 1] - Rm[:, 2, 2]),
         np.maximum(0.0, 1 - Rm[:, 0, 0] + Rm[:, 1, 1] - Rm[:, 2, 2]),
         np.maximum(0.0, 1 - Rm[:, 0, 0] - Rm[:, 1, 1] + Rm[:, 2, 2])]
    q[:, 0] = np.sqrt(m[0]) / 2
    q[:, 1] = np.copysign(np.sqrt(m[1]) / 2, Rm[:, 2, 1] - Rm[:, 1, 2])
    q[:, 2] = np.copysign(np.sqrt(m[2]) / 2, Rm[:, 0, 2] - Rm[:, 2, 0])
    q[:, 3] = np.copysign(np.sqrt(m[3]) / 2, Rm[:, 1, 0] - Rm[:, 0, 1])
    return q / np.linalg.norm(q, axis=1, keepdims=True)


HD = dict(fx=640.0, fy=640.0, cx=640.0, cy=360.0, width=1280, height=720)


def config2(seed=1, n_points=300_000, with_targets=True):
    """Room scene, 300k Gaussians at SH degree 3, one 1280x720 view at a scan pose; L1 RGB +
    0.2 L1 depth against the ray-traced ground truth."""
    scene = room_scene(seed)
    rng = np.random.default_rng(seed + 1)
    scans = rng.uniform(-15.0, 15.0, (8, 2))
    g, pc = lidar_gaussians(scene, rng, scans, n_points)
    cam = look_camera(np.array([scans[0, 0], scans[0, 1], 1.8]), rng.uniform(0, 2 * np.pi),
                      np.deg2rad(-8.0), **HD)
    tr, td = scene.render_gt(cam) if with_targets else (None, None)
    return dict(gaussians=g, cameras=[cam], target_rgb=[tr], target_depth=[td], lambda_depth=0.2,
                scene=scene, points=pc)


def corridor_keyframes(n_keyframes=100, length=200.0, pitch_deg=-8.0):
    """Keyframe cameras every length/n_keyframes metres along the loop, looking ahead."""
    cams = []
    for k in range(n_keyframes):
        s = k * length / n_keyframes
        p, yaw = loop_point(s)
        cams.append(look_camera(np.array([p[0], p[1], 1.8]), yaw, np.deg2rad(pitch_deg), **HD))
    return cams


def sample_views(step, n_keyframes, n_recent=4, n_history=4, recent_frac=0.1):
    """View schedule: n_recent keyframes from the most recent window (last 10% = 20 m of the
    loop) and n_history from the rest, drawn with default_rng(step)."""
    rng = np.random.default_rng(step)
    n_rec = max(n_recent, int(round(recent_frac * n_keyframes)))
    recent = np.arange(n_keyframes - n_rec, n_keyframes)
    hist = np.arange(0, n_keyframes - n_rec)
    return np.concatenate([rng.choice(recent, n_recent, replace=False),
                           rng.choice(hist, n_history, replace=False)])


def config3(seed=2, n_points=1_500_000, n_keyframes=100, target_views=None):
    """Loop corridor: 1.5M Gaussians (SH degree 3) from ring scans every 1 m along a 200 m loop;
    keyframe cameras every 2 m; 8 views per step (4 recent + 4 history).  Targets are
    ray-traced for the keyframe indices in target_views (None = none)."""
    scene = corridor_scene(seed)
    rng = np.random.default_rng(seed + 1)
    scans = np.array([loop_point(s)[0] for s in np.arange(0.0, 200.0, 1.0)])
    g, pc = lidar_gaussians(scene, rng, scans, n_points)
    # segment id: 10 m segments along the loop = the scan that observed the point // 10
    seg = (pc["scan"] // 10).astype(np.int32)
    cams = corridor_keyframes(n_keyframes)
    targets = {}
    if target_views is not None:
        for k in target_views:
            targets[int(k)] = scene.render_gt(cams[int(k)])
    return dict(gaussians=g, cameras=cams, targets=targets, lambda_depth=0.2, scene=scene,
                points=pc, segment_id=seg, n_segments=20)


FHD = dict(fx=960.0, fy=960.0, cx=960.0, cy=540.0, width=1920, height=1080)


def config4b(seed=4, n_points=4_000_000, with_target=True):
    """Loop corridor at 4M Gaussians (SH degree 3) seen by one 1920x1080 keyframe camera
    (f = 960) at the start of the loop; L1 RGB + 0.2 L1 depth against the ray-traced target."""
    scene = corridor_scene(seed)
    rng = np.random.default_rng(seed + 1)
    scans = np.array([loop_point(s)[0] for s in np.arange(0.0, 200.0, 1.0)])
    g, pc = lidar_gaussians(scene, rng, scans, n_points)
    p, yaw = loop_point(0.0)
    cam = look_camera(np.array([p[0], p[1], 1.8]), yaw, np.deg2rad(-8.0), **FHD)
    tgt = scene.render_gt(cam) if with_target else (None, None)
    return dict(gaussians=g, cameras=[cam], target_rgb=[tgt[0]], target_depth=[tgt[1]], lambda_depth=0.2,
                scene=scene)


QHD = dict(fx=320.0, fy=320.0, cx=320.0, cy=180.0, width=640, height=360)


def c5_scene(seed, n_points=100_000, n_scans=8, n_keyframes=24, targets=True):
    """Scene of the initialisation experiment: a room (boxes drawn from the seed) scanned by the
    ring LiDAR from n_scans positions (the scan index is the point's segment), and n_keyframes
    640x360 keyframe cameras at the scan positions with random headings; every 10th keyframe is
    held out from optimisation.  Targets are ray-traced."""
    scene = room_scene(seed)
    rng = np.random.default_rng(seed + 1)
    scans = rng.uniform(-15.0, 15.0, (n_scans, 2))
    pts, surf, nrm, rngs, scan = scene.lidar(rng, scans, int(n_points * 2.5))
    keep = np.sort(rng.choice(pts.shape[0], n_points, replace=False))
    pts, surf, rngs, scan = pts[keep], surf[keep], rngs[keep], scan[keep]
    col = scene.albedo(pts, surf)
    cams = []
    for k in range(n_keyframes):
        p = scans[k % n_scans] + rng.uniform(-1.0, 1.0, 2)
        cams.append(look_camera(np.array([p[0], p[1], 1.8]), rng.uniform(0, 2 * np.pi), np.deg2rad(-8.0), **QHD))
    held = [k for k in range(n_keyframes) if k % 10 == 0]
    train = [k for k in range(n_keyframes) if k % 10 != 0]
    tg = [scene.render_gt(c) for c in cams] if targets else None
    return dict(points=pts.astype(np.float32), colors=col.astype(np.float32), depth=rngs.astype(np.float32),
                segment=scan.astype(np.int32), n_segments=n_scans, cameras=cams, targets=tg, held_out=held,
                train_views=train, scene=scene)
