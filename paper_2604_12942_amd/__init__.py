"""MI355X-native differentiable Gaussian-splatting rasterizer (binding over libgsr.so).

Every step of the path -- projection, binning and radix sort, compositing, the backward, the
pose gradient, the L1 loss and sparse Adam -- runs in the HIP kernels of ``csrc/`` behind the C
ABI of ``include/gsr.h``.  This module only allocates device memory through torch, marshals
pointers and sizes, and enqueues on torch's current stream.  There is no CPU fallback: if
``libgsr.so`` is missing every entry point raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _abi
from ._abi import GsrError, check

PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


def lib():
    return _abi.load()


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Raster:
    """Image size shared by the views of a call plus the screen tile shape (16x16, 8x32, 32x8)."""

    def __init__(self, width, height, tile_w=16, tile_h=16):
        self.width, self.height, self.tile_w, self.tile_h = int(width), int(height), int(tile_w), int(tile_h)
        self.c = _abi.Raster(self.width, self.height, self.tile_w, self.tile_h)
        self.ntx = -(-self.width // self.tile_w)
        self.nty = -(-self.height // self.tile_h)
        self.tiles = self.ntx * self.nty

    def with_tile(self, tw, th):
        return Raster(self.width, self.height, tw, th)


def camera_tensor(cams, device="cuda"):
    """Pack camera dicts (R, t, fx, fy, cx, cy, width, height, z_near, bg) into a device array of
    gsr_camera records (96 bytes each)."""
    arr = (_abi.Camera * len(cams))()
    for k, c in enumerate(cams):
        arr[k].R[:] = [float(v) for v in np.asarray(c["R"], np.float32).ravel()]
        arr[k].t[:] = [float(v) for v in np.asarray(c["t"], np.float32).ravel()]
        arr[k].fx, arr[k].fy, arr[k].cx, arr[k].cy = c["fx"], c["fy"], c["cx"], c["cy"]
        arr[k].z_near = c.get("z_near", 0.2)
        arr[k].bg[:] = [float(v) for v in np.asarray(c.get("bg", (0, 0, 0)), np.float32).ravel()]
        arr[k].width, arr[k].height = int(c["width"]), int(c["height"])
    raw = np.frombuffer(bytes(arr), np.uint8).copy()
    return torch.from_numpy(raw).to(device)


def gaussians_to_device(g, device="cuda"):
    out = {k: torch.as_tensor(np.ascontiguousarray(g[k], np.float32)).to(device) for k in PARAM_NAMES}
    out["sh_degree"] = int(g["sh_degree"])
    return out


_ROWS = dict(means=3, log_scales=3, quats=4, opacity_logits=1)


def _gauss_struct(P, sh_degree):
    n = P["means"].shape[-1]
    if not 0 <= int(sh_degree) <= 3:
        raise GsrError("sh_degree must be 0..3")
    rows = dict(_ROWS, sh=3 * (int(sh_degree) + 1) ** 2)
    for k in PARAM_NAMES:
        t = P[k]
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise GsrError("parameter %s must be a contiguous float32 device tensor" % k)
        if t.numel() != rows[k] * n:
            raise GsrError("parameter %s must hold %d x n values" % (k, rows[k]))
    return _abi.Gaussians(*[P[k].data_ptr() for k in PARAM_NAMES], n, int(sh_degree), 0)


# ------------------------------------------------------------------------------------------
# thin wrappers with the C names
# ------------------------------------------------------------------------------------------

def project(P, sh_degree, cams, n_views, raster, splats=None, tile_info=None):
    n = P["means"].shape[-1]
    dev = P["means"].device
    if splats is None:
        splats = torch.empty(n_views * n * 12, dtype=torch.float32, device=dev)
    if tile_info is None:
        tile_info = torch.empty(4 * n_views * n, dtype=torch.int32, device=dev)
    g = _gauss_struct(P, sh_degree)
    check(lib().gsr_project(C.byref(g), _ptr(cams), n_views, C.byref(raster.c), _ptr(splats), _ptr(tile_info),
                            _stream()), "gsr_project")
    return splats, tile_info


def bin_sort_workspace(n, n_views, capacity, raster):
    return int(lib().gsr_bin_sort_workspace(n, n_views, capacity, C.byref(raster.c)))


def emission(inst_emit, pair_gid, pair_first, n_pairs):
    """gsr_emission struct over four device int32 tensors (see gsr_bin_sort)."""
    return _abi.Emission(_ptr(inst_emit), _ptr(pair_gid), _ptr(pair_first), _ptr(n_pairs))


def _em(em):
    return C.byref(em) if em is not None else None


def bin_sort(tile_info, n, n_views, raster, inst_gid, capacity, tile_ranges, n_instances, ws, tile_order=None,
             em=None):
    check(lib().gsr_bin_sort(_ptr(tile_info), n, n_views, C.byref(raster.c), _ptr(inst_gid), _em(em), capacity,
                             _ptr(tile_ranges), _ptr(n_instances), _ptr(tile_order), _ptr(ws),
                             ws.numel() * ws.element_size(), _stream()), "gsr_bin_sort")


def render_fwd(splats, inst_gid, tile_ranges, cams, n_views, raster, rgb, depth, T_final, last, n_contrib=None,
               tile_order=None, ws=None, capacity=None):
    """Whole tiles (gsr_render_fwd) without ws; with ws (render_fwd_sliced_workspace bytes) and
    the lists' instance capacity, long tiles are composited in depth slices (gsr_render_fwd_sliced)."""
    if ws is None:
        check(lib().gsr_render_fwd(_ptr(splats), _ptr(inst_gid), _ptr(tile_ranges), _ptr(tile_order), _ptr(cams),
                                   n_views, C.byref(raster.c), _ptr(rgb), _ptr(depth), _ptr(T_final), _ptr(last),
                                   _ptr(n_contrib), _stream()), "gsr_render_fwd")
        return
    if n_contrib is not None or capacity is None:
        raise ValueError("the sliced forward takes the instance capacity and counts no contributors")
    check(lib().gsr_render_fwd_sliced(_ptr(splats), _ptr(inst_gid), _ptr(tile_ranges), _ptr(tile_order), _ptr(cams),
                                      n_views, C.byref(raster.c), _ptr(rgb), _ptr(depth), _ptr(T_final), _ptr(last),
                                      capacity, _ptr(ws), ws.numel() * ws.element_size(), _stream()),
          "gsr_render_fwd_sliced")


def render_fwd_sliced_workspace(n_views, raster, capacity):
    return int(lib().gsr_render_fwd_sliced_workspace(n_views, C.byref(raster.c), capacity))


def render_bwd(splats, inst_gid, inst_emit, tile_ranges, cams, n_views, raster, T_final, last, dL_drgb, dL_ddepth,
               dinst, tile_order=None, fwd_ws=None, capacity=0):
    """gsr_render_bwd.  fwd_ws / capacity: the workspace and capacity of the sliced forward that
    produced T_final and last (the long tiles then run their backward in its depth slices); None
    runs whole tiles."""
    check(lib().gsr_render_bwd(_ptr(splats), _ptr(inst_gid), _ptr(inst_emit), _ptr(tile_ranges), _ptr(tile_order),
                               _ptr(cams), n_views, C.byref(raster.c), _ptr(T_final), _ptr(last), _ptr(dL_drgb),
                               _ptr(dL_ddepth), _ptr(dinst), _ptr(fwd_ws),
                               0 if fwd_ws is None else fwd_ws.numel() * fwd_ws.element_size(), int(capacity),
                               _stream()), "gsr_render_bwd")


def render_bwd_l1_workspace(n_views, raster):
    return int(lib().gsr_render_bwd_l1_workspace(n_views, C.byref(raster.c)))


def render_bwd_l1(splats, inst_gid, inst_emit, tile_ranges, cams, n_views, raster, rgb, depth, T_final, last,
                  target_rgb, target_depth, lambda_depth, loss, dinst, ws, tile_order=None, target_index=None,
                  fwd_ws=None, capacity=0):
    """Render backward of the per-pixel L1 loss (gsr_render_bwd_l1); loss is accumulated.  fwd_ws /
    capacity: the workspace and capacity of the sliced forward that produced the images (the long
    tiles then run their backward in its depth slices); None runs whole tiles."""
    check(lib().gsr_render_bwd_l1(_ptr(splats), _ptr(inst_gid), _ptr(inst_emit), _ptr(tile_ranges),
                                  _ptr(tile_order), _ptr(cams), n_views, C.byref(raster.c), _ptr(rgb), _ptr(depth),
                                  _ptr(T_final), _ptr(last), _ptr(target_rgb), _ptr(target_depth),
                                  _ptr(target_index), float(lambda_depth), _ptr(loss), _ptr(dinst), _ptr(ws),
                                  ws.numel() * ws.element_size(), _ptr(fwd_ws),
                                  0 if fwd_ws is None else fwd_ws.numel() * fwd_ws.element_size(), int(capacity),
                                  _stream()), "gsr_render_bwd_l1")


def render_step_workspace(n_views, raster, capacity):
    return int(lib().gsr_render_step_workspace(n_views, C.byref(raster.c), capacity))


def render_step(splats, inst_gid, inst_emit, tile_ranges, cams, n_views, raster, target_rgb, target_depth,
                lambda_depth, rgb, depth, T_final, last, loss, dinst, capacity, ws, tile_order=None,
                target_index=None):
    """Fused forward + L1 loss + backward of every view-tile (gsr_render_step); loss is accumulated."""
    check(lib().gsr_render_step(_ptr(splats), _ptr(inst_gid), _ptr(inst_emit), _ptr(tile_ranges), _ptr(tile_order),
                                _ptr(cams), n_views, C.byref(raster.c), _ptr(target_rgb), _ptr(target_depth),
                                _ptr(target_index), float(lambda_depth), _ptr(rgb), _ptr(depth), _ptr(T_final),
                                _ptr(last), _ptr(loss), _ptr(dinst), capacity, _ptr(ws),
                                ws.numel() * ws.element_size(), _stream()), "gsr_render_step")


def render_fwd_stored_workspace(n_views, raster):
    return int(lib().gsr_render_fwd_stored_workspace(n_views, C.byref(raster.c)))


def render_fwd_stored(splats, inst_gid, tile_ranges, cams, n_views, raster, rgb, depth, T_final, last, n_contrib,
                      contrib_offsets, contrib_ids, n_contrib_total, ws, tile_order=None):
    check(lib().gsr_render_fwd_stored(_ptr(splats), _ptr(inst_gid), _ptr(tile_ranges), _ptr(tile_order), _ptr(cams),
                                      n_views, C.byref(raster.c), _ptr(rgb), _ptr(depth), _ptr(T_final), _ptr(last),
                                      _ptr(n_contrib), _ptr(contrib_offsets), _ptr(contrib_ids), contrib_ids.numel(),
                                      _ptr(n_contrib_total), _ptr(ws), ws.numel() * ws.element_size(), _stream()),
          "gsr_render_fwd_stored")


def render_bwd_stored(splats, inst_gid, inst_emit, tile_ranges, cams, n_views, raster, T_final, n_contrib,
                      contrib_offsets, contrib_ids, dL_drgb, dL_ddepth, dinst, tile_order=None):
    check(lib().gsr_render_bwd_stored(_ptr(splats), _ptr(inst_gid), _ptr(inst_emit), _ptr(tile_ranges),
                                      _ptr(tile_order), _ptr(cams), n_views, C.byref(raster.c), _ptr(T_final),
                                      _ptr(n_contrib), _ptr(contrib_offsets), _ptr(contrib_ids), contrib_ids.numel(),
                                      _ptr(dL_drgb), _ptr(dL_ddepth), _ptr(dinst), _stream()), "gsr_render_bwd_stored")


def pair_grads(dinst, em, tile_info, n, n_views, dsplat):
    check(lib().gsr_pair_grads(_ptr(dinst), _em(em), _ptr(tile_info), n, n_views, _ptr(dsplat), _stream()),
          "gsr_pair_grads")


def project_bwd_workspace(n, n_views):
    return int(lib().gsr_project_bwd_workspace(n, n_views))


def project_bwd(P, sh_degree, cams, n_views, raster, splats, dinst, em, tile_info, grads, dpose, ws,
                segment_id=None, min_segment=0, row_mask=None):
    g = _gauss_struct(P, sh_degree)
    gr = _abi.ParamGrads(*[grads[k].data_ptr() for k in PARAM_NAMES])
    check(lib().gsr_project_bwd(C.byref(g), _ptr(cams), n_views, C.byref(raster.c), _ptr(splats), _ptr(dinst),
                                _em(em), _ptr(tile_info), C.byref(gr), _ptr(dpose), _ptr(segment_id),
                                int(min_segment), _ptr(row_mask), _ptr(ws),
                                ws.numel() * ws.element_size() if ws is not None else 0, _stream()),
          "gsr_project_bwd")


def visible_list_workspace(n):
    return int(lib().gsr_visible_list_workspace(n))


def visible_list(tile_info, n, n_views, out_list, out_count, ws):
    check(lib().gsr_visible_list(_ptr(tile_info), n, n_views, _ptr(out_list), _ptr(out_count), _ptr(ws),
                                 ws.numel() * ws.element_size(), _stream()), "gsr_visible_list")


def visible_list_noalloc(tile_info, n, n_views, out_list, out_count):
    """gsr_visible_list without a workspace (the library's fixed device scratch; n limited to
    gsr_visible_list_noalloc_max())."""
    check(lib().gsr_visible_list_noalloc(_ptr(tile_info), n, n_views, _ptr(out_list), _ptr(out_count), _stream()),
          "gsr_visible_list_noalloc")


def project_bwd_adam(P, sh_degree, cams, n_views, raster, splats, dinst, em, tile_info, m, v, lr, step_dev,
                     dpose, ws,
                     segment_id=None, min_segment=0, row_mask=None, beta1=0.9, beta2=0.999, eps=1e-15,
                     vis_list=None, vis_count=None):
    """Projection backward fused with sparse Adam: P (parameters) is updated in place.
    lr: (means, log_scales, quats, opacity_logits, sh_dc, sh_rest); step_dev: device int32 [1]."""
    g = _gauss_struct(P, sh_degree)
    A = _abi.AdamFused()
    A.m = _abi.ParamGrads(*[m[k].data_ptr() for k in PARAM_NAMES])
    A.v = _abi.ParamGrads(*[v[k].data_ptr() for k in PARAM_NAMES])
    A.lr[:] = [float(x) for x in lr]
    A.beta1, A.beta2, A.eps = beta1, beta2, eps
    A.step = step_dev.data_ptr()
    check(lib().gsr_project_bwd_adam(C.byref(g), _ptr(cams), n_views, C.byref(raster.c), _ptr(splats), _ptr(dinst),
                                     _em(em), _ptr(tile_info), _ptr(vis_list), _ptr(vis_count), _ptr(segment_id),
                                     int(min_segment), C.byref(A), _ptr(dpose),
                                     _ptr(row_mask), _ptr(ws), ws.numel() * ws.element_size(), _stream()),
          "gsr_project_bwd_adam")


def step_prep(cam_pool, view_idx, cams, view_idx32=None, loss=None, step=None, row_mask=None):
    """gsr_step_prep: cams (uint8 [V*96]) = the pool's records (uint8 [S*96]) at view_idx (int64
    [V]); view_idx32 = view_idx as int32; loss = 0; step += 1; row_mask = 0 (each optional)."""
    V = view_idx.numel()
    if cams.numel() != V * _abi.CAMERA_BYTES or cam_pool.numel() % _abi.CAMERA_BYTES:
        raise GsrError("camera records are %d bytes" % _abi.CAMERA_BYTES)
    if view_idx.dtype != torch.int64 or (view_idx32 is not None and view_idx32.dtype != torch.int32):
        raise GsrError("view_idx int64, view_idx32 int32")
    n = row_mask.numel() if row_mask is not None else 0
    check(lib().gsr_step_prep(_ptr(cam_pool), cam_pool.numel() // _abi.CAMERA_BYTES, _ptr(view_idx), V, _ptr(cams),
                              _ptr(view_idx32), _ptr(loss), _ptr(step), _ptr(row_mask), n, _stream()),
          "gsr_step_prep")


def adam_step(groups, rows, row_mask, beta1=0.9, beta2=0.999, eps=1e-15, step=1):
    """groups: list of (param, grad, m, v, lr) float32 [cols, rows] device tensors."""
    G = _abi.AdamGroups()
    if not 1 <= len(groups) <= _abi.MAX_GROUPS:
        raise GsrError("1..8 parameter groups")
    for k, (p, g, m, v, lr) in enumerate(groups):
        cols = p.numel() // rows if rows else 0
        G.param[k], G.grad[k], G.m[k], G.v[k] = p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr()
        G.cols[k] = cols
        G.lr[k] = lr
    G.n_groups = len(groups)
    check(lib().gsr_adam_step(C.byref(G), rows, _ptr(row_mask), beta1, beta2, eps, step, _stream()),
          "gsr_adam_step")


def loss_l1(rgb, depth, target_rgb, target_depth, n_views, raster, lambda_depth, loss, dL_drgb, dL_ddepth,
            target_index=None):
    check(lib().gsr_loss_l1(_ptr(rgb), _ptr(depth), _ptr(target_rgb), _ptr(target_depth), _ptr(target_index),
                            n_views, C.byref(raster.c), lambda_depth, _ptr(loss), _ptr(dL_drgb), _ptr(dL_ddepth),
                            _stream()), "gsr_loss_l1")


def support_mask(T_final, n_views, raster, tau_geo, r_erode, mask=None, count=None):
    """Eq. 7: interior supervision mask [V, H, W] (uint8) and its pixel count per view (int32
    tensor holding uint32) from the final transmittance [V, H, W]."""
    dev = T_final.device
    H, W = raster.c.height, raster.c.width
    if mask is None:
        mask = torch.empty((n_views, H, W), dtype=torch.uint8, device=dev)
    if count is None:
        count = torch.empty(n_views, dtype=torch.int32, device=dev)
    check(lib().gsr_support_mask(_ptr(T_final), n_views, C.byref(raster.c), tau_geo, r_erode, _ptr(mask), _ptr(count),
                                 _stream()), "gsr_support_mask")
    return mask, count


def loss_workspace(n_views, raster):
    return lib().gsr_loss_workspace(n_views, C.byref(raster.c))


def loss(rgb, depth, target_rgb, target_depth, n_views, raster, loss_acc, dL_drgb, dL_ddepth, mask=None, count=None,
         lambda_rgb=1.0, lambda_ssim=0.0, lambda_depth=0.0, target_index=None, ws=None):
    """Eq. 9-12 (masked L1 colour, SSIM, masked L1 depth).  Accumulates into loss_acc (float64
    [1]); overwrites dL_drgb and dL_ddepth.  Returns the workspace (reuse it across calls)."""
    nb = loss_workspace(n_views, raster)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=rgb.device)
    check(lib().gsr_loss(_ptr(rgb), _ptr(depth), _ptr(target_rgb), _ptr(target_depth), _ptr(target_index), n_views,
                         C.byref(raster.c), _ptr(mask), _ptr(count), lambda_rgb, lambda_ssim, lambda_depth,
                         _ptr(loss_acc), _ptr(dL_drgb), _ptr(dL_ddepth), _ptr(ws), ws.numel(), _stream()),
          "gsr_loss")
    return ws


def row_order(means, segment_id=None, order=None, ws=None):
    """Storage order of the map's rows: by segment, then by the Morton code of the mean (see
    gsr_row_order).  Returns order [n] (int32 tensor holding uint32 row indices)."""
    n = means.shape[1]
    dev = means.device
    order = torch.empty(max(1, n), dtype=torch.int32, device=dev) if order is None else order
    nb = lib().gsr_row_order_workspace(n)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(1, nb), dtype=torch.uint8, device=dev)
    check(lib().gsr_row_order(_ptr(means), _ptr(segment_id), n, _ptr(order), _ptr(ws), ws.numel(), _stream()),
          "gsr_row_order")
    return order


def prune_select(opacity_logits, max_logit, max_ratio, segment_id=None, min_segment=0, keep_index=None,
                 n_keep=None, ws=None):
    """Low-opacity pruning selection (Sec. III-C).  Returns (keep_index [n] int32 tensor holding
    uint32 row indices, n_keep [1] device tensor); the first n_keep entries are the survivors."""
    n = opacity_logits.numel()
    dev = opacity_logits.device
    keep_index = torch.empty(max(1, n), dtype=torch.int32, device=dev) if keep_index is None else keep_index
    n_keep = torch.zeros(1, dtype=torch.int32, device=dev) if n_keep is None else n_keep
    nb = lib().gsr_prune_workspace(n)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(1, nb), dtype=torch.uint8, device=dev)
    check(lib().gsr_prune_select(_ptr(opacity_logits), _ptr(segment_id), min_segment, n, max_logit, max_ratio,
                                 _ptr(keep_index), _ptr(n_keep), _ptr(ws), ws.numel(), _stream()), "gsr_prune_select")
    return keep_index, n_keep


def gather_rows(pairs, src_rows, index, n_rows, dst_rows, dst_offset=0):
    """pairs: list of (src, dst) component-major tensors of 4-byte elements ([c, rows] or [rows])."""
    if len(pairs) > _abi.MAX_ROW_GROUPS:
        raise GsrError("at most %d row groups" % _abi.MAX_ROW_GROUPS)
    G = _abi.RowGroups()
    for k, (src, dst) in enumerate(pairs):
        if src.element_size() != 4 or dst.element_size() != 4 or not dst.is_contiguous() or not src.is_contiguous():
            raise GsrError("gather_rows takes contiguous 4-byte tensors")
        G.src[k], G.dst[k] = src.data_ptr(), dst.data_ptr()
        G.cols[k] = src.numel() // src_rows if src_rows else (dst.numel() // dst_rows if dst_rows else 0)
    G.n_groups = len(pairs)
    check(lib().gsr_gather_rows(C.byref(G), src_rows, _ptr(index), n_rows, dst_rows, dst_offset, _stream()),
          "gsr_gather_rows")


def proximity_filter(map_means, new_means, d_min, ws=None):
    """Insertion filter: (keep [M] uint8, keep_index [M] int32, n_keep [1]) for new means [3, M]
    against map means [3, N]."""
    n_map, n_new = map_means.shape[1], new_means.shape[1]
    dev = new_means.device
    keep = torch.empty(max(1, n_new), dtype=torch.uint8, device=dev)
    keep_index = torch.empty(max(1, n_new), dtype=torch.int32, device=dev)
    n_keep = torch.zeros(1, dtype=torch.int32, device=dev)
    nb = lib().gsr_proximity_workspace(n_map, n_new)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(max(1, nb), dtype=torch.uint8, device=dev)
    check(lib().gsr_proximity_filter(_ptr(map_means), n_map, _ptr(new_means), n_new, d_min, _ptr(keep),
                                     _ptr(keep_index), _ptr(n_keep), _ptr(ws), ws.numel(), _stream()),
          "gsr_proximity_filter")
    return keep, keep_index, n_keep


def gicp_prepare(P, sh_degree, segment_id, src_segment, cams, n_cams, d_max, d_corr, state=None):
    """Loop-registration set-up (Sec. III-D, Eq. 13): returns a state dict (source / target row
    lists, counts, stats and the workspace) for gicp_iterate."""
    G = _gauss_struct(P, sh_degree)
    n = G.n
    dev = P["means"].device
    if state is None or state["n"] != n:
        state = dict(n=n, src_index=torch.empty(max(1, n), dtype=torch.int32, device=dev),
                     tgt_index=torch.empty(max(1, n), dtype=torch.int32, device=dev),
                     counts=torch.zeros(2, dtype=torch.int32, device=dev),
                     stats=torch.zeros(40, dtype=torch.float64, device=dev),
                     ws=torch.empty(max(1, lib().gsr_gicp_workspace(n)), dtype=torch.uint8, device=dev))
    state["d_corr"] = float(d_corr)
    check(lib().gsr_gicp_prepare(C.byref(G), _ptr(segment_id), src_segment, _ptr(cams), n_cams, d_max, d_corr,
                                 _ptr(state["src_index"]), _ptr(state["tgt_index"]), _ptr(state["counts"]),
                                 _ptr(state["stats"]), _ptr(state["ws"]), state["ws"].numel(), _stream()),
          "gsr_gicp_prepare")
    return state


def gicp_iterate(P, sh_degree, state, pose, n_iter, corr=None):
    """n_iter Gauss-Newton iterations of Eq. 16 on pose (device float64 [12]: R row-major, t),
    in place; statistics in state["stats"]."""
    G = _gauss_struct(P, sh_degree)
    check(lib().gsr_gicp_iterate(C.byref(G), _ptr(state["src_index"]), _ptr(state["tgt_index"]),
                                 _ptr(state["counts"]), state["d_corr"], _ptr(pose), _ptr(state["stats"]), _ptr(corr),
                                 n_iter, _ptr(state["ws"]), state["ws"].numel(), _stream()), "gsr_gicp_iterate")


def transform_segment(P, sh_degree, segment_id, segment, pose, ws=None):
    """Moves the Gaussians of one segment by pose (device float64 [12]) in place (Sec. III-D)."""
    n = P["means"].shape[1]
    prm = _abi.Params(*[P[k].data_ptr() for k in PARAM_NAMES])
    ws = torch.empty(96, dtype=torch.float64, device=P["means"].device) if ws is None else ws
    check(lib().gsr_transform_segment(C.byref(prm), n, int(sh_degree), _ptr(segment_id), segment, _ptr(pose), _ptr(ws),
                                      _stream()), "gsr_transform_segment")


def transform_cameras(cams, n_cams, pose, mask=None):
    """Moves the flagged cameras (device gsr_camera records) by pose, in place."""
    check(lib().gsr_transform_cameras(_ptr(cams), n_cams, _ptr(mask), _ptr(pose), _stream()), "gsr_transform_cameras")


def fill_u32(t, value):
    check(lib().gsr_fill_u32(_ptr(t), value & 0xFFFFFFFF, t.numel() * t.element_size() // 4, _stream()),
          "gsr_fill_u32")


# ------------------------------------------------------------------------------------------
# initialisation: voxel PCA and the cascade
# ------------------------------------------------------------------------------------------

VOXEL_FIELDS = ("n_voxels", "n_outside", "key", "start", "count", "point_order", "point_voxel", "mu", "evals", "R",
                "s_pca", "trace", "cls", "reliable")


def voxel_pca(points, seed, out=None, point_cov=None, sigma_g=False):
    """Voxel-PCA fitting of points [3, n] (float32 device tensor).  Returns a dict of device
    tensors named like gsr_voxels (voxel arrays sized n, component-major); out reuses one.
    point_cov [6, n] (world covariances) puts them into Eq. 2; with sigma_g the full descriptor
    covariance [21, n] is returned as out["sigma_g"]."""
    n = points.shape[1]
    dev = points.device
    if out is None:
        i32, f32, u8 = torch.int32, torch.float32, torch.uint8
        out = dict(n_voxels=torch.zeros(1, dtype=i32, device=dev), n_outside=torch.zeros(1, dtype=i32, device=dev))
        for k in ("key", "start", "count", "point_order", "point_voxel"):
            out[k] = torch.empty(max(1, n), dtype=i32, device=dev)
        for k, c in (("mu", 3), ("evals", 3), ("R", 9), ("s_pca", 3)):
            out[k] = torch.empty(c, max(1, n), dtype=f32, device=dev)
        out["trace"] = torch.empty(max(1, n), dtype=f32, device=dev)
        out["cls"] = torch.empty(max(1, n), dtype=u8, device=dev)
        out["reliable"] = torch.empty(max(1, n), dtype=u8, device=dev)
        out["_ws"] = torch.empty((int(lib().gsr_voxel_pca_workspace(n)) + 255) // 256 * 64, dtype=i32, device=dev)
    V = _abi.Voxels(*[_ptr(out[k]) for k in VOXEL_FIELDS])
    ws = out["_ws"]
    sd = int(seed) & ((1 << 64) - 1)
    if point_cov is None:
        check(lib().gsr_voxel_pca(_ptr(points.contiguous()), n, sd, C.byref(V), _ptr(ws), ws.numel() * 4, _stream()),
              "gsr_voxel_pca")
        return out
    if sigma_g and out.get("sigma_g") is None:
        out["sigma_g"] = torch.empty(21, max(1, n), dtype=torch.float32, device=points.device)
    check(lib().gsr_voxel_pca_cov(_ptr(points.contiguous()), _ptr(point_cov.contiguous()), n, sd, C.byref(V),
                                  _ptr(out.get("sigma_g") if sigma_g else None), _ptr(ws), ws.numel() * 4, _stream()),
          "gsr_voxel_pca_cov")
    return out


def cascade(points, colors, depth, vox, pred=None, focal=640.0, beta=0.0, segment=None, n_segments=1, sh_degree=0,
            anchored=False):
    """Cascaded initialisation (Eq. 3): returns (params dict of [c, n] float32 tensors, branch).
    anchored: the model branch takes only the predicted axis ratios and anchors them at d / f
    (Eq. 4)."""
    n = points.shape[1]
    dev = points.device
    K = (sh_degree + 1) ** 2
    f32 = torch.float32
    P = dict(means=torch.empty(3, n, dtype=f32, device=dev), log_scales=torch.empty(3, n, dtype=f32, device=dev),
             quats=torch.empty(4, n, dtype=f32, device=dev), opacity_logits=torch.empty(n, dtype=f32, device=dev),
             sh=torch.empty(3 * K, n, dtype=f32, device=dev))
    branch = torch.empty(max(1, n), dtype=torch.uint8, device=dev)
    ws = torch.empty((int(lib().gsr_cascade_workspace(n_segments if segment is not None else 1)) + 255) // 256 * 64,
                     dtype=torch.int32, device=dev)
    V = _abi.Voxels(*[_ptr(vox[k]) for k in VOXEL_FIELDS])
    O = _abi.Params(*[_ptr(P[k]) for k in PARAM_NAMES])
    fn = lib().gsr_cascade_anchored if anchored else lib().gsr_cascade
    check(fn(_ptr(points.contiguous()), _ptr(colors.contiguous()), _ptr(depth.contiguous()), _ptr(segment),
             int(n_segments), n, C.byref(V), _ptr(pred), float(focal), float(beta), sh_degree, C.byref(O), _ptr(branch),
             _ptr(ws), ws.numel() * 4, _stream()), "gsr_cascade")
    return P, branch[:n]


def voxel_targets(P, vox, cov_t=None, o_t=None, has=None):
    """Per-voxel training targets (gsr_voxel_targets) of the Gaussians P (one per point of vox's
    cloud): (cov_t [6, n], o_t [n], has [n] uint8)."""
    n = P["log_scales"].shape[1]
    dev = P["log_scales"].device
    cov_t = torch.empty(6, max(1, n), dtype=torch.float32, device=dev) if cov_t is None else cov_t
    o_t = torch.empty(max(1, n), dtype=torch.float32, device=dev) if o_t is None else o_t
    has = torch.empty(max(1, n), dtype=torch.uint8, device=dev) if has is None else has
    prm = _abi.Params(None, _ptr(P["log_scales"].contiguous()), _ptr(P["quats"].contiguous()),
                      _ptr(P["opacity_logits"].contiguous()), None)
    V = _abi.Voxels(*[_ptr(vox[k]) for k in VOXEL_FIELDS])
    check(lib().gsr_voxel_targets(C.byref(prm), n, C.byref(V), _ptr(cov_t), _ptr(o_t), _ptr(has), _stream()),
          "gsr_voxel_targets")
    return cov_t, o_t, has


def pointnet_weight_count():
    return int(lib().gsr_pointnet_weight_count())


def pointnet_forward(points, vox, weights, y=None):
    """Point-network prediction [8, n] for the voxels of voxel_pca(points)."""
    n = points.shape[1]
    if y is None:
        y = torch.zeros(8, max(1, n), dtype=torch.float32, device=points.device)
    V = _abi.Voxels(*[_ptr(vox[k]) for k in VOXEL_FIELDS])
    check(lib().gsr_pointnet_fwd(_ptr(points), n, C.byref(V), _ptr(weights), _ptr(y), _stream()), "gsr_pointnet_fwd")
    return y


def pointnet_backward(points, vox, weights, cov_t, o_t, tmask, inv_count, grad, loss, blocks=512, ws=None):
    """Training-loss gradient of the point network into grad (flat layout); loss (float64 [1]) is
    accumulated.  Returns the workspace for reuse."""
    n = points.shape[1]
    if ws is None:
        ws = torch.empty((int(lib().gsr_pointnet_bwd_workspace(blocks)) + 3) // 4, dtype=torch.float32,
                         device=points.device)
    V = _abi.Voxels(*[_ptr(vox[k]) for k in VOXEL_FIELDS])
    check(lib().gsr_pointnet_bwd(_ptr(points), n, C.byref(V), _ptr(weights), _ptr(cov_t), _ptr(o_t), _ptr(tmask),
                                 float(inv_count), int(blocks), _ptr(grad), _ptr(loss), _ptr(ws), ws.numel() * 4,
                                 _stream()), "gsr_pointnet_bwd")
    return ws


# ------------------------------------------------------------------------------------------
# rasterizer state: buffers sized once, grown on demand
# ------------------------------------------------------------------------------------------

class Rasterizer:
    """Owns the device buffers of one (n Gaussians, V views, raster) configuration and runs the
    forward and backward of the hot path through the C ABI."""

    def __init__(self, n, n_views, raster, capacity=None, device="cuda", mode="recompute"):
        """mode: "recompute" (the backward re-walks each tile's list) or "stored" (the forward
        keeps every pixel's list of composited Gaussians for the backward)."""
        if mode not in ("recompute", "stored"):
            raise ValueError("mode must be 'recompute' or 'stored'")
        self.n, self.V, self.raster, self.device, self.mode = int(n), int(n_views), raster, device, mode
        VN = self.V * self.n
        f32, i32 = torch.float32, torch.int32
        self.splats = torch.empty(VN * 12, dtype=f32, device=device)
        self.tile_info = torch.empty(4 * VN, dtype=i32, device=device)
        self.tile_ranges = torch.empty(2 * self.V * raster.tiles, dtype=i32, device=device)
        self.tile_order = torch.empty(self.V * raster.tiles, dtype=i32, device=device)
        self.n_instances = torch.zeros(1, dtype=i32, device=device)
        P = raster.width * raster.height
        self.rgb = torch.empty(self.V, 3, raster.height, raster.width, dtype=f32, device=device)
        self.depth = torch.empty(self.V, raster.height, raster.width, dtype=f32, device=device)
        self.T_final = torch.empty(self.V, raster.height, raster.width, dtype=f32, device=device)
        self.last = torch.empty(self.V, raster.height, raster.width, dtype=i32, device=device)
        self.pair_gid = torch.empty(max(1, VN), dtype=i32, device=device)
        self.pair_first = torch.empty(max(1, VN), dtype=i32, device=device)
        self.n_pairs = torch.zeros(1, dtype=i32, device=device)
        self.pose_ws = torch.empty(max(1, project_bwd_workspace(self.n, self.V) // 8), dtype=torch.float64,
                                   device=device)
        self.dpose = torch.zeros(self.V, 6, dtype=torch.float64, device=device)
        self.keep_dsplat = False  # tests: keep the per-pair screen-space gradients
        self._alloc_instances(capacity if capacity else max(1 << 16, 4 * VN))
        if mode == "stored":
            npx = self.V * raster.width * raster.height
            self.n_contrib = torch.empty(npx, dtype=i32, device=device)
            self.contrib_offsets = torch.empty(npx, dtype=i32, device=device)
            self.n_contrib_total = torch.zeros(1, dtype=i32, device=device)
            self.store_ws = torch.empty((render_fwd_stored_workspace(self.V, raster) + 255) // 256 * 64, dtype=i32,
                                        device=device)
            self.contrib_ids = torch.empty(max(1 << 16, 16 * npx), dtype=i32, device=device)

    def _alloc_instances(self, cap):
        self.capacity = int(min(cap, (1 << 32) - 2))
        self.inst_gid = torch.empty(self.capacity, dtype=torch.int32, device=self.device)
        self.inst_emit = torch.empty(self.capacity, dtype=torch.int32, device=self.device)
        self.dinst = torch.empty(self.capacity * _abi.SPLAT_GRAD_FLOATS, dtype=torch.float32, device=self.device)
        self.em = emission(self.inst_emit, self.pair_gid, self.pair_first, self.n_pairs)
        wsb = bin_sort_workspace(self.n, self.V, self.capacity, self.raster)
        self.bin_ws = torch.empty((wsb + 255) // 256 * 64, dtype=torch.int32, device=self.device)
        # the fused step's workspace begins with the sliced forward's, so one buffer serves both
        wsf = max(render_fwd_sliced_workspace(self.V, self.raster, self.capacity),
                  render_step_workspace(self.V, self.raster, self.capacity))
        self.fwd_ws = torch.empty((wsf + 255) // 256 * 64, dtype=torch.int32, device=self.device)
        self.fwd_sliced = False  # whether fwd_ws holds the slice results of the last sliced forward

    def project(self, P, sh_degree, cams):
        """gsr_project into this rasterizer's buffers (remembered, so that a bin/sort whose
        instances overflowed the capacity can project again after growing it)."""
        self._proj_args = (P, sh_degree, cams)
        project(P, sh_degree, cams, self.V, self.raster, self.splats, self.tile_info)

    def forward(self, P, sh_degree, cams, check_capacity=True, sliced=True):
        """project -> bin/sort -> render; returns (rgb, depth, T_final) views of the buffers.
        sliced=False composites every tile whole (gsr_render_fwd) instead of cutting long tiles
        into depth slices (gsr_render_fwd_sliced)."""
        self.project(P, sh_degree, cams)
        self.bin(check_capacity)
        if self.mode == "stored":
            self.render_stored(cams, check_capacity)
        else:
            ws = self.fwd_ws if sliced else None
            render_fwd(self.splats, self.inst_gid, self.tile_ranges, cams, self.V, self.raster, self.rgb, self.depth,
                       self.T_final, self.last, tile_order=self.tile_order, ws=ws, capacity=self.capacity)
        # the sliced forward leaves in fwd_ws what the backward of its slices starts from
        self.fwd_sliced = self.mode != "stored" and sliced
        return self.rgb, self.depth, self.T_final

    def render_stored(self, cams, check_capacity=True):
        def run():
            render_fwd_stored(self.splats, self.inst_gid, self.tile_ranges, cams, self.V, self.raster, self.rgb,
                              self.depth, self.T_final, self.last, self.n_contrib, self.contrib_offsets,
                              self.contrib_ids, self.n_contrib_total, self.store_ws, tile_order=self.tile_order)
        run()
        if check_capacity:
            total = int(self.n_contrib_total.item()) & 0xFFFFFFFF
            if total > self.contrib_ids.numel():
                self.contrib_ids = torch.empty(int(total * 1.25) + 1024, dtype=torch.int32, device=self.device)
                run()

    def contributors(self):
        """Stored mode: number of stored (pixel, Gaussian) entries of the last forward."""
        return int(self.n_contrib_total.item()) & 0xFFFFFFFF

    def bin(self, check_capacity=True):
        """gsr_bin_sort.  An overflow of the instance capacity empties the frame (see gsr_bin_sort);
        with check_capacity the buffers then grow and the projection and binning run again."""
        def run():
            bin_sort(self.tile_info, self.n, self.V, self.raster, self.inst_gid, self.capacity, self.tile_ranges,
                     self.n_instances, self.bin_ws, self.tile_order, self.em)
        run()
        if check_capacity and self.overflowed():
            self._alloc_instances(int(self.instances() * 1.25) + 1024)
            P, sh_degree, cams = self._proj_args
            project(P, sh_degree, cams, self.V, self.raster, self.splats, self.tile_info)
            run()

    def overflowed(self):
        """Whether the last bin/sort needed more instances than the capacity (synchronises)."""
        return self.instances() > self.capacity

    def instances(self):
        return int(self.n_instances.item()) & 0xFFFFFFFF

    def backward(self, P, sh_degree, cams, dL_drgb, dL_ddepth, grads, want_pose=True, segment_id=None,
                 min_segment=0, row_mask=None):
        """render bwd -> project bwd; parameter gradients are accumulated into grads."""
        self.render_backward(cams, dL_drgb, dL_ddepth)
        if self.keep_dsplat:
            self.dsplat_copy = self.screen_grads()
        project_bwd(P, sh_degree, cams, self.V, self.raster, self.splats, self.dinst, self.em, self.tile_info, grads, self.dpose if want_pose else None, self.pose_ws, segment_id, min_segment,
                    row_mask)
        return self.dpose

    def render_backward(self, cams, dL_drgb, dL_ddepth):
        """The compositing backward alone (instance records in self.dinst)."""
        gd = dL_ddepth.contiguous() if dL_ddepth is not None else None
        if self.mode == "stored":
            render_bwd_stored(self.splats, self.inst_gid, self.inst_emit, self.tile_ranges, cams, self.V,
                              self.raster, self.T_final, self.n_contrib, self.contrib_offsets, self.contrib_ids,
                              dL_drgb.contiguous(), gd, self.dinst, tile_order=self.tile_order)
        else:
            render_bwd(self.splats, self.inst_gid, self.inst_emit, self.tile_ranges, cams, self.V, self.raster,
                       self.T_final, self.last, dL_drgb.contiguous(), gd, self.dinst, tile_order=self.tile_order,
                       fwd_ws=self.fwd_ws if self.fwd_sliced else None, capacity=self.capacity)

    def screen_grads(self):
        """Per-pair screen-space gradients [V*n*10] of the last backward."""
        out = torch.empty(self.V * self.n * _abi.SPLAT_GRAD_FLOATS, dtype=torch.float32, device=self.device)
        pair_grads(self.dinst, self.em, self.tile_info, self.n, self.V, out)
        return out


class _RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rast, sh_degree, cams, pose_delta, means, log_scales, quats, opacity_logits, sh):
        P = dict(means=means.contiguous(), log_scales=log_scales.contiguous(), quats=quats.contiguous(),
                 opacity_logits=opacity_logits.contiguous(), sh=sh.contiguous())
        rgb, depth, Tf = rast.forward(P, sh_degree, cams)
        ctx.rast, ctx.sh_degree, ctx.cams = rast, sh_degree, cams
        ctx.P = P
        ctx.save_for_backward(means, log_scales, quats, opacity_logits, sh)
        alpha = 1.0 - Tf
        ctx.mark_non_differentiable(alpha)
        return rgb.clone(), depth.clone(), alpha

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha):
        rast = ctx.rast
        P = ctx.P
        grads = {k: torch.zeros_like(P[k]) for k in PARAM_NAMES}
        if g_rgb is None:
            g_rgb = torch.zeros_like(rast.rgb)
        dpose = rast.backward(P, ctx.sh_degree, ctx.cams, g_rgb, g_depth, grads, want_pose=True)
        return (None, None, None, dpose.to(torch.float32).clone(), grads["means"], grads["log_scales"],
                grads["quats"], grads["opacity_logits"], grads["sh"])


def rasterize(rast, means, log_scales, quats, opacity_logits, sh, sh_degree, cams, pose_delta=None):
    """Differentiable render of all views of `rast`.  Returns (rgb [V,3,H,W], depth [V,H,W],
    alpha [V,H,W]).  If pose_delta ([V,6], zeros, requires_grad) is given, its .grad receives the
    se(3) gradient of a left perturbation (rho, phi) at the current poses."""
    if pose_delta is None:
        pose_delta = torch.zeros(rast.V, 6, device=means.device, requires_grad=False)
    return _RasterizeFn.apply(rast, sh_degree, cams, pose_delta, means, log_scales, quats, opacity_logits, sh)
