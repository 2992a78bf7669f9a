"""Global Gaussian-map optimisation step (paper Sec. III-C), batched over keyframe views.

One step: the views chosen for this iteration are projected and binned together, rendered
(colour + depth, Eq. 8), supervised with Eq. 9 (by default the L1 colour + lambda_depth L1 depth
loss over all pixels; optionally inside the interior support mask of Eq. 7 and with the SSIM
term of Eq. 11), differentiated back to every parameter (and the per-view pose), and
the visible Gaussians of the unfrozen segments take a sparse Adam step.  Every stage is a
libgsr kernel on torch's current stream; this class only owns buffers.
"""
from __future__ import annotations

import torch

from . import PARAM_NAMES, Rasterizer, adam_step, loss, loss_l1, support_mask

# learning rates per parameter group: means (m), log-scales, quaternions, opacity logits,
# SH DC, SH rest
DEFAULT_LR = dict(means=5e-4, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh_dc=2.5e-3, sh_rest=1.25e-4)


class MapOptimizer:
    def __init__(self, params, sh_degree, cam_pool, target_rgb, target_depth, raster, n_views, lambda_depth=0.2,
                 lr=None, segment_id=None, min_segment=0, capacity=None, device="cuda", fused=True,
                 lambda_rgb=1.0, lambda_ssim=0.0, support=None, render="two_pass"):
        """params: dict of float32 [c, n] device tensors (optimised in place); cam_pool: device
        uint8 [S*96] gsr_camera records; target_rgb [S,3,H,W], target_depth [S,H,W] (or None).
        support = (tau_geo, r_erode) supervises only inside the interior mask of Eq. 7 computed
        from this step's own render; None uses every pixel.  render: how the per-pixel L1 loss is
        rendered and differentiated: "two_pass" (default) the forward launch, then one launch that
        forms the loss gradient in registers and runs the render backward (gsr_render_bwd_l1);
        "persistent" all of it in one persistent launch (gsr_render_step); "separate" forward, loss
        and backward as three launches.  Only "separate" writes the gradient images g_rgb, g_depth.
        The full loss (mask, SSIM) always runs separately."""
        self.P = params
        self.sh_degree = int(sh_degree)
        self.n = params["means"].shape[1]
        self.V = int(n_views)
        self.raster = raster
        self.cam_pool = cam_pool.view(-1, 96)
        self.target_rgb, self.target_depth = target_rgb, target_depth
        self.lambda_depth = float(lambda_depth)
        self.lambda_rgb, self.lambda_ssim = float(lambda_rgb), float(lambda_ssim)
        self.support = support
        self.lr = dict(DEFAULT_LR, **(lr or {}))
        self.segment_id, self.min_segment = segment_id, int(min_segment)
        self.rast = Rasterizer(self.n, self.V, raster, capacity=capacity, device=device)
        self.grads = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
        self.m = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
        self.v = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
        H, W = raster.height, raster.width
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        self.g_rgb = torch.empty(self.V, 3, H, W, device=device)
        self.g_depth = torch.empty(self.V, H, W, device=device)
        self.full_loss = support is not None or self.lambda_ssim != 0.0 or self.lambda_rgb != 1.0
        if render not in ("two_pass", "persistent", "separate"):
            raise ValueError("render must be 'two_pass', 'persistent' or 'separate'")
        self.render = "separate" if self.full_loss else render
        self.fused_render = self.render == "persistent"
        self.bwd_ws = None
        self.sup_mask = torch.ones(self.V, H, W, dtype=torch.uint8, device=device)
        self.sup_count = torch.zeros(self.V, dtype=torch.int32, device=device)
        from . import loss_workspace
        self.loss_ws = torch.empty(loss_workspace(self.V, raster) if self.full_loss else 1, dtype=torch.uint8,
                                   device=device)
        self.row_mask = torch.zeros(self.n, dtype=torch.uint8, device=device)
        self.view_idx = torch.zeros(self.V, dtype=torch.int64, device=device)
        self.view_idx32 = torch.zeros(self.V, dtype=torch.int32, device=device)
        self.cams = torch.empty(self.V * 96, dtype=torch.uint8, device=device)
        self.fused = fused
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=device)
        from . import visible_list_workspace
        self.vis_list = torch.empty(max(1, self.n), dtype=torch.int32, device=device)
        self.vis_count = torch.zeros(1, dtype=torch.int32, device=device)
        self.vis_ws = torch.empty((visible_list_workspace(self.n) + 3) // 4, dtype=torch.int32, device=device)
        self.t = 0

    def _set_rows(self, P, m, v, segment_id):
        """Adopt new row arrays (after pruning or insertion) and re-size every per-row buffer.
        Captured graphs refer to the old buffers: capture again afterwards."""
        from . import visible_list_workspace
        dev = P["means"].device
        self.P, self.m, self.v, self.segment_id = P, m, v, segment_id
        self.n = P["means"].shape[1]
        self.rast = Rasterizer(self.n, self.V, self.raster, device=dev)
        self.grads = {k: torch.zeros_like(P[k]) for k in PARAM_NAMES}
        self.row_mask = torch.zeros(self.n, dtype=torch.uint8, device=dev)
        self.vis_list = torch.empty(max(1, self.n), dtype=torch.int32, device=dev)
        self.vis_ws = torch.empty((visible_list_workspace(self.n) + 3) // 4, dtype=torch.int32, device=dev)
        self.graphs = []

    def _row_arrays(self):
        rows = {k: self.P[k] for k in PARAM_NAMES}
        rows.update({"m_" + k: self.m[k] for k in PARAM_NAMES})
        rows.update({"v_" + k: self.v[k] for k in PARAM_NAMES})
        if self.segment_id is not None:
            rows["segment_id"] = self.segment_id
        return rows

    def _adopt(self, rows):
        P = dict(self.P)
        P.update({k: rows[k] for k in PARAM_NAMES})
        self._set_rows(P, {k: rows["m_" + k] for k in PARAM_NAMES}, {k: rows["v_" + k] for k in PARAM_NAMES},
                       rows.get("segment_id"))

    def prune(self, min_opacity=0.005, max_ratio=0.05):
        """Low-opacity pruning (Sec. III-C) of the unfrozen segments; Adam moments and segment ids
        follow their rows.  Returns the number of removed Gaussians."""
        from .maintain import prune
        rows, removed = prune(self._row_arrays(), self.P["opacity_logits"], min_opacity, max_ratio,
                              self.segment_id, self.min_segment)
        self._adopt(rows)
        return removed

    def insert(self, new_params, new_segment_id=None, d_min=0.05):
        """Insert new Gaussians (dict of [c, m] tensors) except those within d_min of the map,
        with zero Adam moments.  Returns the number inserted."""
        from .maintain import insert
        new = {k: new_params[k] for k in PARAM_NAMES}
        new.update({"m_" + k: torch.zeros_like(new_params[k]) for k in PARAM_NAMES})
        new.update({"v_" + k: torch.zeros_like(new_params[k]) for k in PARAM_NAMES})
        if self.segment_id is not None:
            if new_segment_id is None:
                raise ValueError("the map has segment ids: give the new rows theirs")
            new["segment_id"] = new_segment_id
        rows, added = insert(self._row_arrays(), new, d_min)
        self._adopt(rows)
        return added

    def reorder(self):
        """Store the rows segment by segment, in Morton order of the means inside a segment, so
        that the rows a step touches lie close together in memory (the rendered images and the
        updates do not depend on the order, up to depth ties).  Returns the order: position j
        holds the former row order[j]."""
        from .maintain import reorder
        rows, order = reorder(self._row_arrays(), self.segment_id)
        self._adopt(rows)
        return order

    def set_views(self, idx):
        """Choose this iteration's keyframes (slots of the camera / target pool).  A device
        tensor is copied on the stream without a host round-trip."""
        if isinstance(idx, torch.Tensor) and idx.is_cuda:
            self.view_idx.copy_(idx)
        else:
            self.view_idx.copy_(torch.as_tensor(idx, dtype=torch.int64), non_blocking=False)

    def _groups(self):
        P, G, M, Vv, lr = self.P, self.grads, self.m, self.v, self.lr
        gs = [(P[k], G[k], M[k], Vv[k], lr[k]) for k in ("means", "log_scales", "quats", "opacity_logits")]
        gs.append((P["sh"][0:3], G["sh"][0:3], M["sh"][0:3], Vv["sh"][0:3], lr["sh_dc"]))
        if P["sh"].shape[0] > 3:
            gs.append((P["sh"][3:], G["sh"][3:], M["sh"][3:], Vv["sh"][3:], lr["sh_rest"]))
        return gs

    def _stage_fns(self, check_capacity):
        """The step as an ordered list of (name, fn): every fn only enqueues device work (no host
        synchronisation when check_capacity is False), so any run of stages can be captured."""
        from . import (project, render_bwd, render_bwd_l1, render_bwd_l1_workspace, render_fwd, render_step,
                       project_bwd, project_bwd_adam, step_prep, visible_list)
        r = self.rast
        if self.render == "two_pass" and self.bwd_ws is None:
            self.bwd_ws = torch.empty((render_bwd_l1_workspace(self.V, self.raster) + 255) // 256 * 64,
                                      dtype=torch.int32, device=self.loss.device)

        def gather():
            # the step's cameras and target slots, the loss sum cleared and, for the fused Adam,
            # its step number advanced and the row mask cleared: one launch
            step_prep(self.cam_pool, self.view_idx, self.cams, self.view_idx32, loss=self.loss,
                      step=self.step_dev if self.fused else None, row_mask=self.row_mask if self.fused else None)

        def proj():
            r.project(self.P, self.sh_degree, self.cams)

        def binsort():
            r.bin(check_capacity)

        def fwd():
            if self.fused_render:
                # forward, loss and backward of every view-tile in one persistent launch
                gd = self.target_depth
                render_step(r.splats, r.inst_gid, r.inst_emit, r.tile_ranges, self.cams, self.V, self.raster,
                            self.target_rgb, gd, self.lambda_depth if gd is not None else 0.0, r.rgb, r.depth,
                            r.T_final, r.last, self.loss, r.dinst, r.capacity, r.fwd_ws, tile_order=r.tile_order,
                            target_index=self.view_idx32)
                r.fwd_sliced = False  # the fused step keeps its own slice results in fwd_ws
                return
            render_fwd(r.splats, r.inst_gid, r.tile_ranges, self.cams, self.V, self.raster, r.rgb, r.depth,
                       r.T_final, r.last, tile_order=r.tile_order, ws=r.fwd_ws, capacity=r.capacity)
            r.fwd_sliced = True

        def loss_stage():
            if self.render == "persistent":
                return
            if self.render == "two_pass":
                return  # the loss and its gradient are formed inside the render backward
            gd = self.g_depth if self.target_depth is not None else None
            if not self.full_loss:
                loss_l1(r.rgb, r.depth, self.target_rgb, self.target_depth, self.V, self.raster, self.lambda_depth,
                        self.loss, self.g_rgb, gd, target_index=self.view_idx32)
                return
            mask = count = None
            if self.support is not None:
                tau, rad = self.support
                mask, count = support_mask(r.T_final, self.V, self.raster, tau, rad, self.sup_mask, self.sup_count)
            loss(r.rgb, r.depth, self.target_rgb, self.target_depth, self.V, self.raster, self.loss, self.g_rgb, gd,
                 mask=mask, count=count, lambda_rgb=self.lambda_rgb, lambda_ssim=self.lambda_ssim,
                 lambda_depth=self.lambda_depth, target_index=self.view_idx32, ws=self.loss_ws)

        def bwd():
            if self.render == "persistent":
                return
            if self.render == "two_pass":
                gd = self.target_depth
                render_bwd_l1(r.splats, r.inst_gid, r.inst_emit, r.tile_ranges, self.cams, self.V, self.raster, r.rgb,
                              r.depth, r.T_final, r.last, self.target_rgb, gd,
                              self.lambda_depth if gd is not None else 0.0, self.loss, r.dinst, self.bwd_ws,
                              tile_order=r.tile_order, target_index=self.view_idx32, fwd_ws=r.fwd_ws,
                              capacity=r.capacity)
                return
            render_bwd(r.splats, r.inst_gid, r.inst_emit, r.tile_ranges, self.cams, self.V, self.raster, r.T_final,
                       r.last, self.g_rgb, self.g_depth if self.target_depth is not None else None, r.dinst,
                       tile_order=r.tile_order, fwd_ws=r.fwd_ws, capacity=r.capacity)

        def pbwd():
            if self.fused:
                lr = self.lr
                visible_list(r.tile_info, self.n, self.V, self.vis_list, self.vis_count, self.vis_ws)
                lrs = (lr["means"], lr["log_scales"], lr["quats"], lr["opacity_logits"], lr["sh_dc"], lr["sh_rest"])
                project_bwd_adam(self.P, self.sh_degree, self.cams, self.V, self.raster, r.splats, r.dinst, r.em,
                                 r.tile_info, self.m, self.v, lrs, self.step_dev, r.dpose, r.pose_ws,
                                 self.segment_id, self.min_segment, self.row_mask, vis_list=self.vis_list,
                                 vis_count=self.vis_count)
            else:
                project_bwd(self.P, self.sh_degree, self.cams, self.V, self.raster, r.splats, r.dinst, r.em,
                            r.tile_info, self.grads, r.dpose, r.pose_ws, self.segment_id, self.min_segment,
                            self.row_mask)

        def adam():
            if not self.fused:
                self.t += 1
                adam_step(self._groups(), self.n, self.row_mask, step=self.t)

        return [("gather", gather), ("project", proj), ("bin_sort", binsort), ("render_fwd", fwd), ("loss", loss_stage),
                ("render_bwd", bwd), ("project_bwd", pbwd), ("adam", adam)]

    STAGES = ("gather", "project", "bin_sort", "render_fwd", "loss", "render_bwd", "project_bwd", "adam")

    def step(self, check_capacity=True, timer=None):
        """One optimisation iteration over the chosen views.  timer(stage) is called after each
        stage (e.g. to record events)."""
        for name, fn in self._stage_fns(check_capacity):
            fn()
            if timer:
                timer(name)
        return self.loss

    def capture(self, split=()):
        """Capture the fused step into HIP graphs, cut before each stage named in split (so that
        events can be recorded between the parts).  The instance capacity is fixed from now on;
        call after at least one eager step.  replay() then runs one step."""
        if not self.fused:
            raise ValueError("graph capture needs the fused step (its Adam step counter lives on the device)")
        fns = self._stage_fns(False)
        self._split = tuple(split)
        cuts = [0] + [self.STAGES.index(c) for c in split] + [len(fns)]
        self.graphs = []
        torch.cuda.synchronize()
        for a, b in zip(cuts[:-1], cuts[1:]):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                for _, fn in fns[a:b]:
                    fn()
            self.graphs.append(g)
        torch.cuda.synchronize()
        return self.graphs

    def replay(self, between=None, check_capacity=True):
        """One step from the captured graphs; between(k) is called after part k (not after the
        last).  A step whose instances overflow the captured capacity changes nothing (the bin/sort
        empties its frame); with check_capacity (one device synchronisation per step) that is
        detected here, the capacity grows, the step is captured again and run again.  Without it
        the caller checks overflowed() itself."""
        for k, g in enumerate(self.graphs):
            if k and between:
                between(k)
            g.replay()
        if check_capacity and self.rast.overflowed():
            self.recapture()
            for g in self.graphs:
                g.replay()
            if self.rast.overflowed():
                raise RuntimeError("instance capacity still too small after regrowing")
        return self.loss

    def overflowed(self):
        """Whether the last step's instances overflowed the capacity (synchronises)."""
        return self.rast.overflowed()

    def recapture(self, headroom=1.25):
        """Grow the instance capacity to headroom x the last required count and capture the step
        again with the same cuts.  The overflowed step left no trace but its Adam step number,
        which is taken back."""
        r = self.rast
        need = r.instances()
        r._alloc_instances(max(int(need * headroom) + 1024, r.capacity))
        self.step_dev -= 1
        self.capture(self._split)


def autotune_tile(make_opt, set_views, shapes=((16, 16), (8, 32), (32, 8)), warm=2, timed=3):
    """Tile-shape autotuner of the batched step: for each shape, make_opt(shape) builds an
    optimiser on the same map; warm eager steps (with capacity checks) size its buffers, then
    `timed` eager steps are timed between two device synchronisations.  set_views(opt, k) selects
    the views of step k (the same k for every shape).  Returns (fastest shape, {shape: s/step}).

    Whole-tile images are bit-identical across the shapes; tiles long enough to be composited in
    depth slices are cut at different list positions under different shapes, so there the images
    (and gradients) of the chosen shape differ from another shape's by float rounding only."""
    import time
    res = {}
    for sh in shapes:
        o = make_opt(sh)
        for k in range(warm):
            set_views(o, k)
            o.step(check_capacity=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(timed):
            set_views(o, warm + k)
            o.step(check_capacity=False)
        torch.cuda.synchronize()
        res[tuple(sh)] = (time.perf_counter() - t0) / timed
        del o
        torch.cuda.empty_cache()
    return min(res, key=res.get), res
