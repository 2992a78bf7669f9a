#!/usr/bin/env python3
"""Throughput of the batched global-map optimisation step on one MI355X.

Workload (the headline configuration): the 200 m loop-corridor LiDAR scene with 1.5M Gaussians
at SH degree 3; every step renders 8 keyframe views at 1280x720 (4 from the recent window, 4
from the history window), takes the L1 colour + 0.2 L1 depth loss against ray-traced targets,
back-propagates to every parameter and the per-view pose, and applies sparse Adam to the
visible Gaussians of the 5 latest segments.  A step is one pass of the whole hot path:
project, bin/sort, render forward, loss, render backward, project backward, Adam.

Prints one JSON line: iterations/s with blends/s, the roofline of the dominant kernel (from HIP
events on the launch stream) and the FP64 oracle timed on host cores as a baseline.
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# without packed FP32 (the library is compiled without packed FP32 instructions):
# 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
FP32_PEAK_NONPACKED_TFLOPS = 78.6
# algorithmic float operations per composited (pixel, Gaussian) pair, plus one exp each (not
# counted): forward 20, backward 45 (the fused step does both)
FLOP_PER_BLEND_FWD = 20
FLOP_PER_BLEND_BWD = 45
# optimiser iterations from the initialisation to the timed (steady) state of the map
STEADY_ITERS = 500
# the kernel each timed stage launches (its name in rocprofv3 kernel traces)
KERNEL_OF_STAGE = dict(project="k_project", bin_sort="gsr_bin_sort (12 kernels)", render_fwd="k_render_fwd",
                       loss="k_loss_l1", render_bwd="k_render_bwd", project_bwd="k_project_bwd")
# HBM bytes per launch of a kernel measured with rocprofv3 FETCH_SIZE / WRITE_SIZE counters on this
# workload, each scaled by the counter's reading for a 256 MiB device copy (fetch x1.9997, write x1.0);
# keyed by (kernel, tile), with the SHA-256 prefix of the kernel's sources at measurement time: a
# figure whose sources have changed since is reported as null.
TRAFFIC = {("k_render_bwd_l1", "8x32"): (2914947201, "37f55fef502d2a0d")}
KERNEL_SOURCES = {"k_render_bwd_l1": ["csrc/gsr_internal.h", "csrc/render.hip"],
                  "k_render_fwd": ["csrc/gsr_internal.h", "csrc/render.hip"],
                  "k_project_bwd": ["csrc/gsr_internal.h", "csrc/project.hip"]}


def traffic_of(kernel, tile):
    """Measured HBM bytes per launch, or None when unmeasured or measured on other sources."""
    import hashlib
    ent = TRAFFIC.get((kernel, tile))
    if ent is None or kernel not in KERNEL_SOURCES:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2604_12942_amd", f), "rb") as fh:
            h.update(fh.read())
    return ent[0] if h.hexdigest()[:16] == ent[1] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--tile", default="auto", help="auto | 16x16 | 8x32 | 32x8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches instead of the captured step")
    ap.add_argument("--no-maintenance", action="store_true",
                    help="skip the pruning / insertion, loop-registration and init-path timing")
    ap.add_argument("--no-full-loss", action="store_true",
                    help="skip the leg with the support mask and the SSIM term in the loss")
    ap.add_argument("--points", type=int, default=1_500_000)
    ap.add_argument("--no-c2", action="store_true", help="skip the one-view 300k-Gaussian room leg")
    ap.add_argument("--no-disc-map", action="store_true",
                    help="skip the step on the flat-disc stand-in map (opacity 0.1)")
    ap.add_argument("--no-init-compare", action="store_true",
                    help="skip the learned vs voxel-PCA init comparison leg (iterations to a PSNR target)")
    ap.add_argument("--contrib-compare", action="store_true",
                    help="instead of the step: stored vs recomputed contributor lists on the 4M-Gaussian 1080p view")
    ap.add_argument("--init-compare", action="store_true",
                    help="instead of the step: iterations to a held-out PSNR target, learned vs voxel-PCA init")
    ap.add_argument("--train-scenes", type=int, default=20)
    ap.add_argument("--test-scenes", type=int, default=5)
    ap.add_argument("--init-iters", type=int, default=3000)
    ap.add_argument("--net-steps", type=int, default=600)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 256 MiB device-to-device copy (reference for HBM byte counters)")
    ap.add_argument("--profile-region", action="store_true",
                    help="launch a marker kernel (torch spin kernel) right before and after the steady-state "
                         "timed steps, so that profiler output can be cut to exactly the timed dispatches")
    return ap.parse_args()


class ProfileRegion:
    """Marks the steady-state timed steps in a profiler trace: a short spin kernel (torch's
    cuda._sleep) is launched on the stream right before the first and right after the last timed
    step, so that a kernel trace or counter run can keep exactly the dispatches in between."""

    def __init__(self, enabled):
        self.enabled = enabled

    def mark(self, stream):
        if self.enabled:
            import torch
            with torch.cuda.stream(stream):
                torch.cuda._sleep(1000)


def _render_target(args):
    scene, cam = args
    return scene.render_gt(cam)


def cascade_map(c, seg, dev, seed=1):
    """Gaussians of the LiDAR points from the voxel-PCA cascade on the GPU (voxel fit, then Eq. 3
    without a model: PCA branch with the per-segment beta of Eq. 5, else the heuristic branch of
    Eq. 6 at the point's range over the keyframes' focal length); higher-order SH from the
    generator (N(0, 0.05^2)) so that the full degree-3 colour work is exercised."""
    import torch

    import paper_2604_12942_amd as gsr
    pc = c["points"]
    pts = torch.from_numpy(np.ascontiguousarray(pc["points"].T)).to(dev)
    col = torch.from_numpy(np.ascontiguousarray(pc["colors"].T)).to(dev)
    depth = torch.from_numpy(np.ascontiguousarray(pc["ranges"])).to(dev)
    vox = gsr.voxel_pca(pts, seed)
    P, _ = gsr.cascade(pts, col, depth, vox, focal=640.0, beta=0.0, segment=seg, n_segments=int(c["n_segments"]),
                       sh_degree=3)
    P["sh"][3:] = torch.from_numpy(c["gaussians"]["sh"][3:]).to(dev)
    torch.cuda.synchronize()
    return P


def build_workload(n_points, workers):
    c = synth.config3(n_points=n_points)
    cams = c["cameras"]
    nk = len(cams)
    # keyframe pool: the 8 most recent keyframes (recent window) and 8 spread over the rest
    recent = list(range(nk - 8, nk))
    history = [int(round(x)) for x in np.linspace(0, nk - 12, 8)]
    pool = recent + history
    with ProcessPoolExecutor(max_workers=workers) as ex:
        tg = list(ex.map(_render_target, [(c["scene"], cams[k]) for k in pool]))
    return c, [cams[k] for k in pool], tg


def views_for_step(step):
    rng = np.random.default_rng(step)
    return np.concatenate([rng.choice(8, 4, replace=False), 8 + rng.choice(8, 4, replace=False)])


def cpu_model():
    """The host CPU's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(c, pool_cams, tg, step_views, n_sample=4):
    """FP64 oracle on n_sample of the 8 views of one step (forward + L1 loss + backward incl. pose,
    over all Gaussians at full resolution), scaled to a whole step."""
    import oracle
    oracle.lib()
    g = c["gaussians"]
    t0 = time.perf_counter()
    blends = 0
    for k in step_views[:n_sample]:
        cam = pool_cams[k]
        r = oracle.render(g, cam)
        blends += int(r["n"].sum())
        _, gC, gD = oracle.l1_loss(r["rgb"], r["depth"], tg[k][0], tg[k][1], 0.2)
        oracle.render_bwd(g, cam, gC, gD)
    dt = time.perf_counter() - t0
    V = len(step_views)
    return dict(value=round(n_sample / (V * dt), 5), unit="iters/s", blends_per_s=round(blends / dt, 1),
                cores=oracle.num_threads(), kind="oracle",
                nproc=len(os.sched_getaffinity(0)), cpu_model=cpu_model(),
                sample="%d of the %d views of one step (forward + L1 loss + backward incl. pose, all %d Gaussians, "
                       "%dx%d), %.1f s, scaled to %d views" % (n_sample, V, g["means"].shape[1], pool_cams[0]["width"],
                                                              pool_cams[0]["height"], dt, V))


def oracle_step_time(g, cam, trgb, tdep, lam):
    """The FP64 oracle's fwd + bwd step of one view (full render, L1 loss, backward with pose):
    (seconds, blends)."""
    import oracle
    oracle.lib()
    t0 = time.perf_counter()
    r = oracle.render(g, cam)
    _, gC, gD = oracle.l1_loss(r["rgb"], r["depth"], trgb, tdep if lam > 0 else None, lam)
    oracle.render_bwd(g, cam, gC, gD if lam > 0 else None)
    return time.perf_counter() - t0, int(r["n"].sum())


def cpu_baseline_configs():
    """The oracle's one-view step on C1 (2,000 Gaussians SH0, 128x96, its own target) and C2 (the
    300k-Gaussian room, one 1280x720 view, a constant grey target: the timing does not depend on
    it).  C4b's is in the --contrib-compare line.  Returns {config: {iters_per_s, blends_per_s, ...}}."""
    out = {}
    for name, c in (("c1", synth.config1()), ("c2", synth.config2(with_targets=False))):
        g, cam = c["gaussians"], c["cameras"][0]
        H, W = cam["height"], cam["width"]
        trgb = c["target_rgb"][0] if c["target_rgb"][0] is not None else np.full((3, H, W), 0.5, np.float32)
        tdep = c["target_depth"][0] if c["target_depth"][0] is not None else np.full((H, W), 5.0, np.float32)
        dt, blends = oracle_step_time(g, cam, trgb, tdep, c.get("lambda_depth") or 0.0)
        out[name] = dict(gaussians=int(g["means"].shape[1]), pixels=W * H, iters_per_s=round(1.0 / dt, 4),
                         blends_per_s=round(blends / dt, 1), seconds=round(dt, 2))
        print("cpu baseline %s: %s" % (name, out[name]), file=sys.stderr, flush=True)
    return out


def contrib_compare(a):
    """Forward + backward of one 1920x1080 view over 4M Gaussians in both contributor modes:
    time per iteration and peak device memory (one JSON line)."""
    import torch

    import paper_2604_12942_amd as gsr
    t_gen = time.perf_counter()
    c = synth.config4b()
    print("workload built in %.1f s" % (time.perf_counter() - t_gen), file=sys.stderr, flush=True)
    g, cam = c["gaussians"], c["cameras"][0]
    dev = "cuda"
    n = g["means"].shape[1]
    H, W = cam["height"], cam["width"]
    trgb = torch.from_numpy(c["target_rgb"][0][None]).to(dev)
    tdep = torch.from_numpy(c["target_depth"][0][None]).to(dev)
    ct = gsr.camera_tensor([cam], dev)
    res = {}
    for mode in ("recompute", "stored"):
        torch.cuda.empty_cache()
        P = gsr.gaussians_to_device(g, dev)
        grads = {k: torch.zeros_like(P[k]) for k in gsr.PARAM_NAMES}
        g_rgb = torch.empty(1, 3, H, W, device=dev)
        g_dep = torch.empty(1, H, W, device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        rast = gsr.Rasterizer(n, 1, gsr.Raster(W, H, 16, 16), mode=mode, device=dev)

        def it(check):
            rast.forward(P, g["sh_degree"], ct, check_capacity=check)
            loss.zero_()
            gsr.loss_l1(rast.rgb, rast.depth, trgb, tdep, 1, rast.raster, 0.2, loss, g_rgb, g_dep)
            rast.backward(P, g["sh_degree"], ct, g_rgb, g_dep, grads, want_pose=True)

        it(True)
        torch.cuda.synchronize()
        free0, total = torch.cuda.mem_get_info()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        reps = max(3, min(a.steps, 10))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            it(False)
        e1.record()
        torch.cuda.synchronize()
        mode_bytes = 0
        if mode == "stored":
            mode_bytes = sum(t.numel() * t.element_size()
                             for t in (rast.contrib_ids, rast.n_contrib, rast.contrib_offsets, rast.store_ws))
        res[mode] = dict(ms_per_iter=round(e0.elapsed_time(e1) / reps, 3),
                         peak_allocated_bytes=int(torch.cuda.max_memory_allocated()),
                         resident_before_bytes=int(base), device_used_bytes=int(total - free0),
                         list_bytes=int(mode_bytes),
                         contributors=rast.contributors() if mode == "stored" else None,
                         instances=rast.instances(), loss=float(loss.item()))
        del rast, P, grads
    out = {"metric": "contributor storage: fwd+bwd ms/iter and peak memory, 4M Gaussians, 1920x1080",
           "config": {"workload": "loop corridor, %d Gaussians SH3, one 1920x1080 view, L1 rgb + 0.2 L1 depth" % n,
                      "tile": "16x16"},
           "data": "synthetic", "dtype": "f32", "modes": res}
    if not a.no_cpu_baseline:
        # the FP64 oracle's step of the same view (host cores, one step)
        import oracle
        dt, blends = oracle_step_time(g, cam, c["target_rgb"][0], c["target_depth"][0], 0.2)
        out["cpu_baseline"] = dict(value=round(1.0 / dt, 5), unit="iters/s", blends_per_s=round(blends / dt, 1),
                                   cores=oracle.num_threads(), nproc=len(os.sched_getaffinity(0)),
                                   cpu_model=cpu_model(), kind="oracle",
                                   sample="one full fwd + L1 loss + bwd (with pose) step, %.1f s" % dt)
    print(json.dumps(out), flush=True)


def _c5_scene(seed):
    c = synth.c5_scene(seed)
    c.pop("scene")
    return c


def init_compare_scenes(a):
    """The training and test scenes of the init comparison, built in worker processes (before the
    GPU is used in this process)."""
    t0 = time.perf_counter()
    train_seeds = list(range(100, 100 + a.train_scenes))
    test_seeds = list(range(200, 200 + a.test_scenes))
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        data = dict(zip(train_seeds + test_seeds, ex.map(_c5_scene, train_seeds + test_seeds)))
    print("init-compare scenes built in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    return train_seeds, test_seeds, data


def init_compare(a, scenes=None):
    """Iterations to a held-out PSNR target from the learned-cascade init versus the voxel-PCA
    cascade (beta grid-tuned on the training scenes), identical optimiser settings.  Returns the
    summary dict."""
    train_seeds, test_seeds, data = scenes if scenes is not None else init_compare_scenes(a)
    import torch

    import paper_2604_12942_amd as gsr
    from paper_2604_12942_amd import learned_init as li
    from paper_2604_12942_amd.optimize import MapOptimizer

    dev = "cuda"
    t0 = time.perf_counter()
    V = 4
    every = 25

    def run(c, P, iters, seed, curve=True):
        cams = c["cameras"]
        W, H = cams[0]["width"], cams[0]["height"]
        raster = gsr.Raster(W, H, 16, 16)
        tv, hv = c["train_views"], c["held_out"]
        trgb = torch.from_numpy(np.stack([c["targets"][k][0] for k in tv])).to(dev)
        tdep = torch.from_numpy(np.stack([c["targets"][k][1] for k in tv])).to(dev)
        hrgb = torch.from_numpy(np.stack([c["targets"][k][0] for k in hv])).to(dev)
        opt = MapOptimizer(P, 3, gsr.camera_tensor([cams[k] for k in tv], dev), trgb, tdep, raster, V,
                           lambda_depth=0.2, device=dev)
        held = gsr.Rasterizer(P["means"].shape[1], len(hv), raster, device=dev)
        hcams = gsr.camera_tensor([cams[k] for k in hv], dev)
        rng = np.random.default_rng(seed)
        sched = torch.from_numpy(np.stack([rng.choice(len(tv), V, replace=False) for _ in range(iters)])).to(dev)
        out = []

        def psnr():
            rgb, _, _ = held.forward(P, 3, hcams)
            mse = torch.mean((rgb.clamp(0, 1) - hrgb) ** 2)
            return float(10 * torch.log10(1.0 / mse).item())

        if curve:
            out.append((0, psnr()))
        for it in range(iters):
            opt.set_views(sched[it])
            opt.step(check_capacity=True)
            if curve and (it + 1) % every == 0:
                out.append((it + 1, psnr()))
        return out if curve else psnr()

    def init(c, seed, weights=None, beta=0.0):
        sc = li.SceneInit(c["points"], c["colors"], c["depth"], c["segment"], c["n_segments"], seed=seed, device=dev)
        P, br = sc.gaussians(weights=weights, beta=beta)
        return sc, P, br

    # 1. the voxel-PCA judge: Eq. 5's beta grid-tuned on training scenes (held-out PSNR at 1000 its)
    grid = [0.25, 0.35, 0.5, 0.7, 1.0]
    tune = {}
    for b in grid:
        vals = []
        for sd in train_seeds[:5]:
            sc, P, _ = init(data[sd], sd, beta=b)
            vals.append(run(data[sd], P, min(1000, a.init_iters), sd, curve=False))
        tune[b] = float(np.mean(vals))
    beta = max(grid, key=lambda b: tune[b])
    print("beta tuning %s -> %.2f" % (tune, beta), file=sys.stderr, flush=True)
    # 2. training targets: train scenes optimised from the tuned PCA init
    scenes, targets = [], []
    for sd in train_seeds:
        sc, P, _ = init(data[sd], sd, beta=beta)
        run(data[sd], P, a.init_iters, sd, curve=False)
        scenes.append(sc)
        targets.append(sc.targets(P))
    print("train maps optimised (%.1f s)" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    # 3. the point network
    weights = li.init_weights(0, dev)
    net_loss = li.train_pointnet(scenes, targets, weights, a.net_steps,
                                 log=lambda it, l: print("net step %d loss %.4f" % (it, l), file=sys.stderr,
                                                         flush=True))
    # 4. test scenes: identical optimiser, views and iterations from both inits
    res = []
    for sd in test_seeds:
        c = data[sd]
        _, PA, bA = init(c, sd, beta=beta)
        curveA = run(c, PA, a.init_iters, 1000 + sd)
        _, PB, bB = init(c, sd, weights=weights)
        curveB = run(c, PB, a.init_iters, 1000 + sd)
        target = curveA[-1][1] - 0.25
        first = lambda cur: next((it for it, p in cur if p >= target), None)
        at = lambda cur, it: next((p for i, p in cur if i == it), None)
        bc = np.bincount(bB.cpu().numpy(), minlength=3)
        res.append(dict(seed=sd, psnr_target=round(target, 3), iters_pca=first(curveA), iters_learned=first(curveB),
                        psnr_pca={k: round(at(curveA, k), 3) for k in (0, 100, 300, 1000, a.init_iters)
                                  if at(curveA, k) is not None},
                        psnr_learned={k: round(at(curveB, k), 3) for k in (0, 100, 300, 1000, a.init_iters)
                                      if at(curveB, k) is not None},
                        branch_counts_learned=dict(model=int(bc[0]), pca=int(bc[1]), heuristic=int(bc[2]))))
        print("test %d: %s" % (sd, res[-1]), file=sys.stderr, flush=True)
    wins = sum(1 for r in res if r["iters_learned"] is not None and
               (r["iters_pca"] is None or r["iters_learned"] < r["iters_pca"]))
    ratios = [r["iters_learned"] / r["iters_pca"] for r in res if r["iters_learned"] and r["iters_pca"]]
    return {"metric": "iterations to held-out PSNR target, learned vs voxel-PCA init",
           "config": {"workload": "room scenes, 100k LiDAR points, 24 keyframes 640x360 (every 10th held out), "
                                  "4 views per iteration, SH3", "train_scenes": len(train_seeds),
                      "test_scenes": len(test_seeds), "iterations": a.init_iters, "net_steps": a.net_steps},
           "data": "synthetic", "beta_tuned": beta, "beta_grid_psnr_1000": {str(k): round(v, 3) for k, v in tune.items()},
           "net_final_loss": round(net_loss, 5), "tests": res, "learned_wins": wins,
           "mean_iter_ratio": round(float(np.mean(ratios)), 4) if ratios else None,
           "gate": bool(wins >= max(1, (4 * len(res) + 4) // 5) and ratios and float(np.mean(ratios)) < 1.0),
           "mean_psnr_gain_at": {str(k): round(float(np.mean([r["psnr_learned"][k] - r["psnr_pca"][k] for r in res
                                                              if k in r["psnr_learned"] and k in r["psnr_pca"]])), 3)
                                 for k in (0, 100, 300, 1000, a.init_iters)},
           "seconds": round(time.perf_counter() - t0, 1)}


FULL_LOSS = dict(lambda_rgb=0.8, lambda_ssim=0.2, support=(0.5, 2))
# algorithmic HBM bytes per pixel of the full loss stage: support mask (T 4, mask 1), masked L1
# (rgb 12, targets 16, depth 4, mask 1, gradients 16), SSIM forward (images 24, mask 1, three
# derivative maps per channel 36), SSIM backward (maps 36, images 24, mask 1, gradient RMW 24)
FULL_LOSS_BYTES_PER_PX = 5 + 49 + 61 + 85
# float operations per pixel of the stage's dominant kernels: the SSIM forward (separable 11-tap
# filters of five moments, the SSIM map and its three derivative maps, about 190 per channel) and
# backward (the filters' adjoints and the chain rule, about 110 per channel), three channels
FULL_LOSS_FLOP_PER_PX = 3 * (190 + 110)


def full_loss_leg(make_opt, sv, a, tile, stages, stream, pixels):
    """The same step with the supervision mask (Eq. 7) and the SSIM term (Eq. 11) in the loss:
    captured-step throughput, per-stage times and the loss stage's HBM roofline."""
    import torch
    o = make_opt(tile, **FULL_LOSS)
    for s in range(a.warmup):
        sv(o, s)
        o.step(check_capacity=True)
    k = max(3, min(a.steps, 10))
    stage_ms = {st: 0.0 for st in stages}
    for s in range(k):
        evs = {}

        def mark(name, evs=evs):
            e = torch.cuda.Event(enable_timing=True)
            e.record(stream)
            evs[name] = e

        e0 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sv(o, s)
        o.step(check_capacity=False, timer=mark)
        torch.cuda.synchronize()
        prev = e0
        for st in stages:
            stage_ms[st] += prev.elapsed_time(evs[st]) / k
            prev = evs[st]
    o.capture()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(a.steps):
        sv(o, a.warmup + s)
        o.replay(check_capacity=False)
    torch.cuda.synchronize()
    if o.overflowed():
        print("instance capacity exceeded in the timed region (full loss)", file=sys.stderr)
        sys.exit(3)
    ms = 1000.0 * (time.perf_counter() - t0) / a.steps
    ach = FULL_LOSS_BYTES_PER_PX * pixels / (stage_ms["loss"] / 1000.0) / 1e9
    fl = FULL_LOSS_FLOP_PER_PX * pixels / (stage_ms["loss"] / 1000.0) / 1e12
    res = dict(lambda_rgb=FULL_LOSS["lambda_rgb"], lambda_ssim=FULL_LOSS["lambda_ssim"], lambda_depth=0.2,
               tau_geo=FULL_LOSS["support"][0], r_erode=FULL_LOSS["support"][1], iters_per_s=round(1000.0 / ms, 3),
               ms_per_step=round(ms, 3), stage_ms={st: round(v, 4) for st, v in stage_ms.items()},
               mask_pixels=int(o.sup_count.sum().item()), loss_last=float(o.loss.item()),
               loss_roofline=dict(bound="alu", achieved=round(fl, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                                  frac=round(fl / FP32_PEAK_TFLOPS, 4),
                                  frac_of_nonpacked_peak=round(fl / FP32_PEAK_NONPACKED_TFLOPS, 4),
                                  flop_per_pixel=FULL_LOSS_FLOP_PER_PX,
                                  hbm_achieved_GBps=round(ach, 1), hbm_frac=round(ach / HBM_PEAK_GBS, 4),
                                  kernels="k_support_mask, k_loss_masked, k_ssim_fwd, k_ssim_bwd",
                                  alg_bytes_per_launch=FULL_LOSS_BYTES_PER_PX * pixels))
    print("full loss: %s" % res, file=sys.stderr, flush=True)
    del o
    torch.cuda.empty_cache()
    return res


# map maintenance readings: at most 5 % of the rows pruned per call; insertion filter radius 5 cm.
# The timed pruning call uses opacity threshold 0.2, above the initial opacity of every row, so
# that all rows of the unfrozen segments are candidates and the budget binds (the selection's
# worst case: the full candidate sort); the reading for training is 0.005.
PRUNE_MIN_OPACITY, PRUNE_MAX_RATIO, INSERT_D_MIN = 0.2, 0.05, 0.05


def maintenance_leg(g, seg, min_seg, dev, reps=5):
    """Pruning (selection + compaction of parameters, Adam moments and segment ids) and the
    proximity-filtered insertion of a re-scanned segment, on the full map; kernel times from HIP
    events on the launch stream, median over reps."""
    import torch

    import paper_2604_12942_amd as gsr
    from paper_2604_12942_amd.maintain import _gather_all
    P = gsr.gaussians_to_device(g, dev)
    n = P["means"].shape[1]
    rows = {k: P[k] for k in gsr.PARAM_NAMES}
    rows.update({"m_" + k: torch.zeros_like(P[k]) for k in gsr.PARAM_NAMES})
    rows.update({"v_" + k: torch.zeros_like(P[k]) for k in gsr.PARAM_NAMES})
    rows["segment_id"] = seg
    floats_per_row = sum(t.numel() // n for t in rows.values())
    # new segment: 40k means re-observing mapped surface (2 cm jitter) and 20k off the map
    rng = np.random.default_rng(11)
    src = torch.from_numpy(rng.integers(0, n, 60_000)).to(dev)
    jit = torch.from_numpy(np.concatenate([rng.normal(0, 0.02, (3, 40_000)), rng.normal(0, 0.5, (3, 20_000))],
                                          axis=1).astype(np.float32)).to(dev)
    new_means = (P["means"][:, src] + jit).contiguous()
    stream = torch.cuda.current_stream()
    import math
    max_logit = math.log(PRUNE_MIN_OPACITY / (1 - PRUNE_MIN_OPACITY))

    def timed(fn):
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            out = fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)), out

    t_sel, (keep, n_keep) = timed(lambda: gsr.prune_select(P["opacity_logits"], max_logit, PRUNE_MAX_RATIO, seg,
                                                           min_seg))
    k = int(n_keep.item())
    dst = {name: torch.empty(tuple(t.shape[:-1]) + (k,), dtype=t.dtype, device=dev) for name, t in rows.items()}
    t_cmp, _ = timed(lambda: _gather_all([(rows[nm], dst[nm]) for nm in rows], n, keep, k, k, 0))
    t_prox, (keep_new, idx, n_new) = timed(lambda: gsr.proximity_filter(P["means"], new_means, INSERT_D_MIN))
    kn = int(n_new.item())
    # storage order (segment-major, Morton inside a segment) and the move of every row into it
    t_ord, order = timed(lambda: gsr.row_order(P["means"], seg))
    dst2 = {name: torch.empty_like(t) for name, t in rows.items()}
    t_mv, _ = timed(lambda: _gather_all([(rows[nm], dst2[nm]) for nm in rows], n, order, n, n, 0))
    b_cmp = 2 * 4 * floats_per_row * k + 4 * k
    res = dict(rows=n, floats_per_row=floats_per_row, min_opacity=PRUNE_MIN_OPACITY, max_ratio=PRUNE_MAX_RATIO,
               removed=n - k, prune_select_ms=round(t_sel, 4), compaction_ms=round(t_cmp, 4),
               compaction_roofline=dict(bound="hbm", achieved=round(b_cmp / (t_cmp / 1e3) / 1e9, 1), peak=HBM_PEAK_GBS,
                                        unit="GB/s", frac=round(b_cmp / (t_cmp / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                                        alg_bytes_per_launch=b_cmp),
               insert_candidates=int(new_means.shape[1]), insert_d_min=INSERT_D_MIN, inserted=kn,
               proximity_ms=round(t_prox, 4), row_order_ms=round(t_ord, 4), row_move_ms=round(t_mv, 4))
    print("maintenance: %s" % res, file=sys.stderr, flush=True)
    del P, rows, dst, dst2
    torch.cuda.empty_cache()
    return res


def loop_leg(c, seg, dev, reps=3):
    """Loop registration on the full map: the last segment (closing the loop) against what the first
    four keyframes see within 30 m, from a drifted initial pose (1 deg of yaw about the target
    set's centre, 0.2 m across the corridor, 0.1 m up); then the corrected pose is propagated to the segment's Gaussians.  The map itself is
    consistent, so the ideal correction is the identity; the displacement it leaves is measured over
    the source means paired in the last linearisation.  Kernel times from HIP events."""
    import torch

    import paper_2604_12942_amd as gsr
    from paper_2604_12942_amd import loop
    g = c["gaussians"]
    P = gsr.gaussians_to_device(g, dev)
    src_seg = int(c["segment_id"].max())
    cams = gsr.camera_tensor(c["cameras"][:4], dev)
    yaw = np.deg2rad(1.0)
    R0 = np.array([[np.cos(yaw), -np.sin(yaw), 0.0], [np.sin(yaw), np.cos(yaw), 0.0], [0.0, 0.0, 1.0]])
    stream = torch.cuda.current_stream()
    state = gsr.gicp_prepare(P, g["sh_degree"], seg, src_seg, cams, 4, loop.D_MAX, loop.D_CORR)
    nt = int(state["counts"][1].item())
    centre = g["means"][:, state["tgt_index"][:nt].cpu().numpy()].astype(np.float64).mean(axis=1)
    # drift: 1 deg of yaw about the centre of the target set, 0.2 m across and 0.1 m up
    t0 = centre - R0 @ centre + np.array([0.0, 0.2, 0.1])
    rec = []
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record(stream)
        state = gsr.gicp_prepare(P, g["sh_degree"], seg, src_seg, cams, 4, loop.D_MAX, loop.D_CORR, state)
        e[1].record(stream)
        pose = torch.tensor(np.concatenate([R0.ravel(), t0]), dtype=torch.float64, device=dev)
        corr = torch.empty(P["means"].shape[1], dtype=torch.int32, device=dev)
        gsr.gicp_iterate(P, g["sh_degree"], state, pose, 30, corr=corr)
        e[2].record(stream)
        torch.cuda.synchronize()
        rec.append((e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])))
    st = state["stats"].cpu().numpy()
    its = int(st[37])
    prep = float(np.median([r[0] for r in rec]))
    itm = float(np.median([r[1] for r in rec]))
    pz = pose.cpu().numpy()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    gsr.transform_segment(P, g["sh_degree"], seg, src_seg, pose)
    e1.record(stream)
    torch.cuda.synchronize()
    count = int(st[29])
    # RMS motion under the estimated pose of the source means paired in the last linearisation
    # (the overlap with the target set)
    ns = int(state["counts"][0].item())
    sm = g["means"][:, c["segment_id"] == src_seg].astype(np.float64)
    paired = corr[:ns].cpu().numpy() >= 0
    sm = sm[:, paired]
    disp = float(np.sqrt(np.mean(np.sum((pz[:9].reshape(3, 3) @ sm + pz[9:, None] - sm) ** 2, axis=0))))
    disp0 = float(np.sqrt(np.mean(np.sum((R0 @ sm + t0[:, None] - sm) ** 2, axis=0))))
    ang = float(np.degrees(np.arccos(np.clip((np.trace(pz[:9].reshape(3, 3)) - 1) / 2, -1, 1))))
    res = dict(rows=int(P["means"].shape[1]), n_src=int(state["counts"][0].item()),
               n_tgt=int(state["counts"][1].item()), d_max=loop.D_MAX, d_corr=loop.D_CORR, iterations=its,
               converged=bool(st[36]), correspondences=count, mean_cost=round(float(st[27]) / max(count, 1), 5),
               accepted=bool(st[36] and count >= loop.MIN_CORR and st[27] / max(count, 1) < loop.ACCEPT_COST),
               prepare_ms=round(prep, 4), iterations_ms=round(itm, 4), ms_per_iteration=round(itm / max(its, 1), 4),
               initial_displacement_rms_m=round(disp0, 4), final_displacement_rms_m=round(disp, 5),
               final_rotation_deg=round(ang, 5),
               propagate_ms=round(e0.elapsed_time(e1), 4))
    print("loop registration: %s" % res, file=sys.stderr, flush=True)
    del P, state
    torch.cuda.empty_cache()
    return res


# point network forward: per voxel 32 rows x (3x64 + 64x64 + 64x64) and the 76x64 + 64x8 head
PN_FLOP_PER_VOXEL = 2 * 32 * (192 + 4096 + 4096) + 2 * (4864 + 512)
BF16_PEAK_TFLOPS = 2500.0


def init_leg(dev, reps=5):
    """The initialisation path on a batch of 200k occupied voxels with 32 LiDAR-like points each
    (6.4M points): voxel PCA (isotropic, and with per-point LiDAR covariances in Eq. 2), the point
    network forward and the cascade, timed with HIP events (median of reps)."""
    import torch

    import paper_2604_12942_amd as gsr
    from paper_2604_12942_amd import learned_init as li
    pts, cols, org, rngs = synth.voxel_batch(0)
    n = pts.shape[0]
    cov = torch.from_numpy(np.ascontiguousarray(synth.lidar_point_cov(pts, org).T)).to(dev)
    t = torch.from_numpy(np.ascontiguousarray(pts.T)).to(dev)
    col = torch.from_numpy(np.ascontiguousarray(cols.T)).to(dev)
    depth = torch.from_numpy(rngs).to(dev)
    w = li.init_weights(0, dev)
    stream = torch.cuda.current_stream()

    def timed(fn):
        ts = []
        out = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            out = fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts)), out

    vox = gsr.voxel_pca(t, 1)
    t_pca, _ = timed(lambda: gsr.voxel_pca(t, 1, out=vox))
    nv = int(vox["n_voxels"].item())
    rel_iso = int(vox["reliable"][:nv].sum().item())
    t_cov, _ = timed(lambda: gsr.voxel_pca(t, 1, out=vox, point_cov=cov, sigma_g=True))
    rel_cov = int(vox["reliable"][:nv].sum().item())
    pred = torch.zeros(8, n, dtype=torch.float32, device=dev)  # allocated outside the timed calls
    t_pn, _ = timed(lambda: gsr.pointnet_forward(t, vox, w, y=pred))
    t_cas, _ = timed(lambda: gsr.cascade(t, col, depth, vox, pred=pred, focal=640.0, beta=0.0, sh_degree=3))
    ach = PN_FLOP_PER_VOXEL * nv / (t_pn / 1e3) / 1e12
    res = dict(points=n, voxels=nv, reliable_isotropic=rel_iso, reliable_point_cov=rel_cov,
               voxel_pca_ms=round(t_pca, 4), voxel_pca_point_cov_ms=round(t_cov, 4), pointnet_fwd_ms=round(t_pn, 4),
               cascade_ms=round(t_cas, 4),
               pointnet_roofline=dict(bound="mfma", achieved=round(ach, 2), peak=BF16_PEAK_TFLOPS, unit="TFLOP/s",
                                      frac=round(ach / BF16_PEAK_TFLOPS, 5), flop_per_voxel=PN_FLOP_PER_VOXEL))
    print("init path: %s" % res, file=sys.stderr, flush=True)
    del vox, t, cov
    torch.cuda.empty_cache()
    return res


def render_modes_leg(make_opt, sv, tile, params, stages, stream, first_step, k=5):
    """The same steps (same map, same views) with the render, L1 loss and render backward as three
    launches, as two (the loss inside the render backward) and as one persistent launch: the sum
    of those stages' times in ms per step (HIP events on the launch stream, eager steps)."""
    import torch
    res = {}
    for mode in ("separate", "two_pass", "persistent"):
        o = make_opt(tile, params=params, render=mode)
        for s in range(3):
            sv(o, first_step + s)
            o.step(check_capacity=True)
        tot = 0.0
        for s in range(k):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

            def mark(name, ev=ev):
                if name == "bin_sort":
                    ev[0].record(stream)
                elif name == "render_bwd":
                    ev[1].record(stream)

            sv(o, first_step + 3 + s)
            o.step(check_capacity=False, timer=mark)
            torch.cuda.synchronize()
            tot += ev[0].elapsed_time(ev[1])
        res[mode] = round(tot / k, 4)
        del o
        torch.cuda.empty_cache()
    print("render modes (fwd + loss + bwd ms/step): %s" % res, file=sys.stderr, flush=True)
    return res


def disc_map_leg(params, make_opt, tile, fit_capacity, measure, sampled_workload, a):
    """The same captured step (same views, same loss, same optimiser) on a simpler map of the same
    corridor: one flat disc per LiDAR point, aligned with the surface (in-plane scale about 0.1 m,
    normal scale 2 cm), opacity 0.1 everywhere, as generated (no optimiser iterations before the
    timed steps).  Reports iterations/s, the stages, the workload and the render backward's rate
    by the blend count."""
    import torch
    o = make_opt(tile, params=params)
    del params
    fit_capacity(o, 0, a.warmup)
    k = max(3, min(a.steps, 10))
    r = measure(o, a.warmup, k)
    wl = sampled_workload(o, r)
    # the timed steps' own render-backward times when that stage dominates, else the stage pass's
    bwd_ms = wl["dom_ms"] if r["dom"] == "render_bwd" else r["stage_ms"]["render_bwd"]
    kname = "k_render_bwd_l1" if o.render == "two_pass" else "k_render_bwd"
    ach = wl["blends"] * FLOP_PER_BLEND_BWD / (bwd_ms / 1000.0) / 1e12
    out = dict(workload="loop corridor, %d flat-disc Gaussians SH3 at opacity 0.1 as generated, 8 views 1280x720 per "
                        "step, the headline's step" % int(o.P["means"].shape[1]),
               iters_per_s=round(1000.0 / r["ms_per_step"], 3), ms_per_step=round(r["ms_per_step"], 3),
               stage_ms={kk: round(v, 4) for kk, v in r["stage_ms"].items()},
               blends_per_step=int(round(wl["blends"])), instances_per_step=int(round(wl["M"])),
               visible_pairs_per_step=int(round(wl["Nv"])),
               render_bwd_roofline=dict(kernel=kname, bound="alu", stage_ms=round(bwd_ms, 4),
                                        achieved=round(ach, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                                        frac=round(ach / FP32_PEAK_TFLOPS, 4),
                                        frac_of_nonpacked_peak=round(ach / FP32_PEAK_NONPACKED_TFLOPS, 4),
                                        flop_per_unit=FLOP_PER_BLEND_BWD))
    print("disc map: %s" % json.dumps(out), file=sys.stderr, flush=True)
    del o
    torch.cuda.empty_cache()
    return out


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Device-to-device copy of 1 GiB: (read + write bytes) / time in GB/s, the measured ceiling the
    step's algorithmic bytes are also compared with."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) / 1000.0) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return gbs


def c2_leg(a, dev, steps=20):
    """The one-view room configuration: 300k Gaussians at SH degree 3 from the voxel-PCA cascade,
    one 1280x720 view, the step (forward + L1 rgb + 0.2 L1 depth + backward + sparse Adam),
    captured; iterations/s, blends/s and the render forward + loss + backward share of the step."""
    import torch

    import paper_2604_12942_amd as gsr
    from paper_2604_12942_amd.optimize import MapOptimizer
    c = synth.config2()
    cam = c["cameras"][0]
    W, H = cam["width"], cam["height"]
    seg = torch.zeros(c["gaussians"]["means"].shape[1], dtype=torch.int32, device=dev)
    P = cascade_map(dict(c, n_segments=1), seg, dev)
    trgb = torch.from_numpy(c["target_rgb"][0][None]).to(dev)
    tdep = torch.from_numpy(c["target_depth"][0][None]).to(dev)
    o = MapOptimizer(P, 3, gsr.camera_tensor([cam], dev), trgb, tdep, gsr.Raster(W, H, 16, 16), 1, lambda_depth=0.2,
                     device=dev)
    o.set_views([0])
    for _ in range(3):
        o.step(check_capacity=True)
    o.capture(split=("render_fwd", "project_bwd"))
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rend = 0.0
    for _ in range(steps):
        e[0].record(stream)

        def between(k):
            if k == 1:
                e[1].record(stream)
            elif k == 2:
                e[2].record(stream)

        o.replay(between=between, check_capacity=False)
        torch.cuda.synchronize()
        rend += e[1].elapsed_time(e[2])
    ms = 1000.0 * (time.perf_counter() - t0) / steps
    if o.overflowed():
        print("instance capacity exceeded in the C2 leg", file=sys.stderr)
        sys.exit(3)
    r = o.rast
    ncon = torch.empty(1, H, W, dtype=torch.int32, device=dev)
    gsr.render_fwd(r.splats, r.inst_gid, r.tile_ranges, o.cams, 1, o.raster, r.rgb, r.depth, r.T_final, r.last,
                   ncon, tile_order=r.tile_order)
    torch.cuda.synchronize()
    blends = int(ncon.sum().item())
    rend /= steps
    ach = blends * (FLOP_PER_BLEND_FWD + FLOP_PER_BLEND_BWD) / (rend / 1000.0) / 1e12
    res = dict(workload="room, %d Gaussians SH3 from the voxel-PCA cascade, one 1280x720 view, L1 rgb + 0.2 L1 "
                        "depth, sparse Adam, captured step (%s render)" % (P["means"].shape[1], o.render),
               iters_per_s=round(1000.0 / ms, 3), ms_per_step=round(ms, 4), blends_per_step=blends,
               blends_per_s=round(blends / (ms / 1000.0), 1), instances=r.instances(),
               render_fwd_loss_bwd_ms=round(rend, 4),
               render_roofline=dict(bound="alu", achieved=round(ach, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                                    frac=round(ach / FP32_PEAK_TFLOPS, 4), flop_per_blend=FLOP_PER_BLEND_FWD +
                                    FLOP_PER_BLEND_BWD))
    print("C2: %s" % res, file=sys.stderr, flush=True)
    del o
    torch.cuda.empty_cache()
    return res


def main():
    a = parse()
    if a.init_compare:
        print(json.dumps(init_compare(a)), flush=True)
        return
    if a.contrib_compare:
        if a.gpus != 1:
            print("bench.py measures one GPU only", file=sys.stderr)
            sys.exit(2)
        contrib_compare(a)
        return
    if a.copy_calibration:
        import torch
        x = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}))
        return
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    t_gen = time.perf_counter()
    workers = min(8, os.cpu_count() or 1)
    c, pool_cams, tg = build_workload(a.points, workers)
    ic_scenes = None if a.no_init_compare else init_compare_scenes(a)
    print("workload built in %.1f s" % (time.perf_counter() - t_gen), file=sys.stderr, flush=True)

    import torch

    import paper_2604_12942_amd as gsr
    from paper_2604_12942_amd.optimize import MapOptimizer, autotune_tile

    dev = "cuda"
    n = c["gaussians"]["means"].shape[1]
    V = 8
    H, W = pool_cams[0]["height"], pool_cams[0]["width"]
    trgb = torch.from_numpy(np.stack([x[0] for x in tg])).to(dev)
    tdep = torch.from_numpy(np.stack([x[1] for x in tg])).to(dev)
    cam_pool = gsr.camera_tensor(pool_cams, dev)
    seg = torch.from_numpy(c["segment_id"]).to(dev)
    min_seg = int(c["n_segments"]) - 5
    # the map: the LiDAR points initialised on the GPU by the voxel-PCA cascade (Eq. 3, 5, 6)
    P0 = cascade_map(c, seg, dev)
    g = {k: P0[k].cpu().numpy() for k in gsr.PARAM_NAMES}
    g["sh_degree"] = 3

    def make_opt(tile, params=None, **kw):
        P = {k: (params or P0)[k].clone() for k in gsr.PARAM_NAMES}
        raster = gsr.Raster(W, H, *tile)
        o = MapOptimizer(P, 3, cam_pool, trgb, tdep, raster, V, lambda_depth=0.2, segment_id=seg,
                         min_segment=min_seg, device=dev, **kw)
        o.reorder()  # the map's rows in storage order: by segment, Morton order inside a segment
        return o

    # the view schedule of every step, resident on the device (no host round-trip per step)
    n_main = a.warmup + 2 * (10 + max(a.steps, 10)) + STEADY_ITERS + 16
    sched = torch.from_numpy(np.stack([views_for_step(s) for s in range(n_main)] +
                                      [views_for_step(10_000 + s) for s in range(2)] +
                                      [views_for_step(10_100 + s) for s in range(3)])).to(dev)
    row_of = {s: s for s in range(n_main)}
    row_of.update({10_000 + s: n_main + s for s in range(2)})
    row_of.update({10_100 + s: n_main + 2 + s for s in range(3)})

    def sv(o, step):
        o.set_views(sched[row_of[step]])

    def timed_steps(opt, k, first_step):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(k):
            sv(opt, first_step + s)
            opt.step(check_capacity=False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    # project-written autotuner (package: paper_2604_12942_amd.optimize.autotune_tile)
    shapes = [(16, 16), (8, 32), (32, 8)] if a.tile == "auto" else [tuple(int(x) for x in a.tile.split("x"))]
    if len(shapes) > 1:
        tile, tune = autotune_tile(make_opt, lambda o, s: sv(o, 10_000 + s if s < 2 else 10_100 + s - 2), shapes)
        tune = {"%dx%d" % k: v for k, v in tune.items()}
    else:
        tile, tune = shapes[0], {}
    print("tile autotune (s/step): %s -> %dx%d" % (tune, *tile), file=sys.stderr, flush=True)

    stages = list(MapOptimizer.STAGES)
    stream = torch.cuda.current_stream()

    def staged_steps(o, k, first_step):
        """k eager steps with HIP events on the launch stream after every stage."""
        recs = []
        for s in range(k):
            evs = {}

            def mark(name, evs=evs):
                e = torch.cuda.Event(enable_timing=True)
                e.record(stream)
                evs[name] = e

            e0 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            sv(o, first_step + s)
            o.step(check_capacity=False, timer=mark)
            recs.append((e0, evs))
        return recs

    def worst_views_instances(o):
        """Instances of the heaviest step the view schedule can draw: each pool view's own count
        (the 8 recent, then the 8 history keyframes, binned as one step each), the 4 largest of
        each window summed."""
        fns = dict(o._stage_fns(True))
        T = o.raster.tiles
        per = []
        for half in range(2):
            o.set_views(torch.arange(8 * half, 8 * half + 8, device=dev))
            for name in ("gather", "project", "bin_sort"):
                fns[name]()
            rg = o.rast.tile_ranges.view(V, T, 2).to(torch.int64) & 0xFFFFFFFF
            per.append(sorted((rg[:, :, 1] - rg[:, :, 0]).sum(dim=1).tolist()))
        return sum(per[0][-4:]) + sum(per[1][-4:])

    def fit_capacity(o, first_step, k):
        """k eager steps with capacity checks, then room for 1.3 x the larger of their largest
        instance count and the heaviest step the schedule can draw."""
        m_max = 0
        for s in range(k):
            sv(o, first_step + s)
            o.step(check_capacity=True)
            m_max = max(m_max, o.rast.instances())
        m_max = max(m_max, worst_views_instances(o))
        if o.rast.capacity < int(m_max * 1.3):
            o.rast._alloc_instances(int(m_max * 1.3))

    region = ProfileRegion(a.profile_region)

    def measure(o, first_step, k_timed, profiled=False):
        """Stage breakdown (its own pass), then k_timed captured steps with HIP events on the launch
        stream: around every step (percentiles) and around the dominant kernel's stage.  profiled:
        the timed steps are bracketed by profiler markers."""
        recs = staged_steps(o, max(3, min(k_timed, 10)), first_step)
        torch.cuda.synchronize()
        stage_ms = {k: 0.0 for k in stages}
        for e0, evs in recs:
            prev = e0
            for k in stages:
                stage_ms[k] += prev.elapsed_time(evs[k])
                prev = evs[k]
        stage_ms = {k: v / len(recs) for k, v in stage_ms.items()}
        dom = max(stage_ms, key=stage_ms.get)
        i_dom = stages.index(dom)
        split = (dom,) + ((stages[i_dom + 1],) if i_dom + 1 < len(stages) else ())
        if i_dom == 0:
            split = split[1:]
        o.capture(split=split)
        dom_part = 0 if i_dom == 0 else 1
        m_seen = torch.zeros(k_timed, dtype=torch.int32, device=dev)
        ev_dom, ev_step = [], []
        torch.cuda.synchronize()
        if profiled:
            region.mark(stream)
        t0 = time.perf_counter()
        for s in range(k_timed):
            e_a = torch.cuda.Event(enable_timing=True)
            e_b = torch.cuda.Event(enable_timing=True)
            e_s = torch.cuda.Event(enable_timing=True)
            e_s.record(stream)
            ev_step.append(e_s)
            sv(o, first_step + len(recs) + s)
            if dom_part == 0:
                e_a.record(stream)

            def between(k, e_a=e_a, e_b=e_b):
                if k == dom_part:
                    e_a.record(stream)
                elif k == dom_part + 1:
                    e_b.record(stream)

            o.replay(between=between, check_capacity=False)
            if dom_part + 1 == len(o.graphs):
                e_b.record(stream)
            m_seen[s:s + 1].copy_(o.rast.n_instances)
            ev_dom.append((e_a, e_b))
        e_end = torch.cuda.Event(enable_timing=True)
        e_end.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if profiled:
            region.mark(stream)
            torch.cuda.synchronize()
        m_all = m_seen.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
        if m_all.max() > o.rast.capacity:
            print("instance capacity exceeded in the timed region", file=sys.stderr)
            sys.exit(3)
        per_step = [a_.elapsed_time(b_) for a_, b_ in zip(ev_step, ev_step[1:] + [e_end])]
        dom_per_step = [e_a.elapsed_time(e_b) for e_a, e_b in ev_dom]
        return dict(ms_per_step=1000.0 * wall / k_timed, per_step=per_step, stage_ms=stage_ms, dom=dom,
                    dom_ms=sum(dom_per_step) / k_timed, dom_per_step=dom_per_step,
                    first_timed=first_step + len(recs), last_step=first_step + len(recs) + k_timed - 1)

    def workload_stats(o, step):
        """Blends, instances, visible pairs and updated rows (visible in a view and in one of the
        unfrozen segments) of one step's views on the current map."""
        sv(o, step)
        dict(o._stage_fns(False))["gather"]()  # the step's cameras
        r = o.rast
        ncon = torch.empty(V, H, W, dtype=torch.int32, device=dev)
        r.project(o.P, o.sh_degree, o.cams)
        r.bin(True)
        gsr.render_fwd(r.splats, r.inst_gid, r.tile_ranges, o.cams, V, o.raster, r.rgb, r.depth, r.T_final, r.last,
                       ncon, tile_order=r.tile_order)
        torch.cuda.synchronize()
        vis = r.tile_info.view(4, V, -1)[0] > 0
        upd = vis.any(dim=0)
        if o.segment_id is not None:
            upd &= o.segment_id >= o.min_segment
        return dict(blends=int(ncon.sum().item()), M=r.instances(), Nv=int(vis.sum().item()),
                    Nu=int(upd.sum().item()))

    def sampled_workload(o, r, n_sample=10):
        """The workload of up to n_sample of the timed steps, evenly spaced: the means of their
        blends, instances, visible pairs and updated rows, with the mean of the same steps'
        dominant-stage times.  Each step's views are rendered again after the timed run, so the map
        is the one the run ended with: it moved on by at most that many optimiser iterations."""
        k = len(r["dom_per_step"])
        idx = sorted(set(int(round(x)) for x in np.linspace(0, k - 1, min(n_sample, k))))
        ws = [workload_stats(o, r["first_timed"] + s) for s in idx]
        out = {key: float(np.mean([w[key] for w in ws])) for key in ("blends", "M", "Nv", "Nu")}
        out["dom_ms"] = float(np.mean([r["dom_per_step"][s] for s in idx]))
        out["steps"] = len(idx)
        return out

    opt = make_opt(tile)
    fit_capacity(opt, 0, a.warmup)
    # the map as initialised: a shorter timed run
    k_init = max(3, min(a.steps, 10))
    at_init = measure(opt, a.warmup, k_init)
    wl_init = sampled_workload(opt, at_init)
    # steady state: STEADY_ITERS optimiser iterations from the initialisation, then the timed run
    s0 = at_init["last_step"] + 1
    for s in range(STEADY_ITERS):
        sv(opt, s0 + s)
        opt.replay(check_capacity=True)
    s0 += STEADY_ITERS
    fit_capacity(opt, s0, 3)
    res = measure(opt, s0 + 3, a.steps, profiled=True)
    wl = sampled_workload(opt, res)
    # the roofline pairs the sampled steps' dominant-stage times with their own workload
    stage_ms, dom, dom_ms, ms_per_step = res["stage_ms"], res["dom"], wl["dom_ms"], res["ms_per_step"]
    blends, M, Nv, Nu = (int(round(wl[k])) for k in ("blends", "M", "Nv", "Nu"))
    g = {k: opt.P[k].cpu().numpy() for k in gsr.PARAM_NAMES}  # the map the CPU baseline renders
    g["sh_degree"] = 3
    c = dict(c, gaussians=g, disc_gaussians=c["gaussians"])

    # eager step time without events (for reference)
    eager_ms = 1000.0 * timed_steps(opt, max(3, min(a.steps, 10)), 0)
    use_graph = True

    Pf = 59
    P = W * H
    T = opt.raster.tiles
    B = dict(project=V * 12 * n + (4 * Pf - 12) * Nv + 52 * Nv,
             bin_sort=8 * Nv + 12 * M + 24 * M + 8 * M + 8 * V * T,
             render_fwd=44 * M + 24 * V * P,
             render_bwd=44 * M + 40 * V * P + 40 * Nv,
             project_bwd=Nv * (40 + 4 * Pf + 8 * Pf),
             adam=Nu * 4 * Pf * 8)
    B_alg = sum(B.values())
    step_s = ms_per_step / 1000.0
    fused = opt.fused_render
    render_mode = opt.render
    kname = "k_render_step" if (fused and dom == "render_fwd") else KERNEL_OF_STAGE[dom]
    if opt.render == "two_pass" and dom == "render_bwd":
        kname = "k_render_bwd_l1"
    if dom in ("render_fwd", "render_bwd"):
        fpb = (FLOP_PER_BLEND_FWD + FLOP_PER_BLEND_BWD) if (fused and dom == "render_fwd") else \
            (FLOP_PER_BLEND_FWD if dom == "render_fwd" else FLOP_PER_BLEND_BWD)
        fl = blends * fpb
        ach = fl / (dom_ms / 1000.0) / 1e12
        roof = dict(bound="alu", achieved=round(ach, 3), peak=FP32_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=round(ach / FP32_PEAK_TFLOPS, 4), traffic=traffic_of(kname, "%dx%d" % tile),
                    frac_of_nonpacked_peak=round(ach / FP32_PEAK_NONPACKED_TFLOPS, 4),
                    kernel=kname, launch_ms=round(dom_ms, 4), units_per_launch=blends, unit_kind="blend",
                    flop_per_unit=fpb, sampled_steps=wl["steps"], launch_ms_all_steps=round(res["dom_ms"], 4))
    else:
        ach = B[dom] / (dom_ms / 1000.0) / 1e9
        roof = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=traffic_of(kname, "%dx%d" % tile),
                    kernel=kname, launch_ms=round(dom_ms, 4), alg_bytes_per_launch=B[dom], sampled_steps=wl["steps"],
                    launch_ms_all_steps=round(res["dom_ms"], 4))
    pct = np.percentile(np.asarray(res["per_step"]), [10, 50, 90])
    init_pct = np.percentile(np.asarray(at_init["per_step"]), [10, 50, 90])
    at_init_out = dict(iters_per_s=round(1000.0 / at_init["ms_per_step"], 3),
                       ms_per_step=round(at_init["ms_per_step"], 3),
                       step_ms_p10_p50_p90=[round(float(x), 4) for x in init_pct],
                       stage_ms={k: round(v, 4) for k, v in at_init["stage_ms"].items()},
                       blends_per_step=int(round(wl_init["blends"])), instances_per_step=int(round(wl_init["M"])),
                       blends_per_s=round(wl_init["blends"] / (at_init["ms_per_step"] / 1000.0), 1))

    loss_last = float(opt.loss.item())
    modes = render_modes_leg(make_opt, sv, tile, opt.P, stages, stream, s0)
    disc = None
    if not a.no_disc_map:
        disc = disc_map_leg(gsr.gaussians_to_device(c["disc_gaussians"], dev), make_opt, tile, fit_capacity, measure,
                            sampled_workload, a)
    maint = loopr = initr = None
    if not a.no_maintenance:
        maint = maintenance_leg(g, seg, min_seg, dev)
        loopr = loop_leg(c, seg, dev)
        initr = init_leg(dev)
    full = None
    if not a.no_full_loss:
        del opt
        torch.cuda.empty_cache()
        full = full_loss_leg(make_opt, sv, a, tile, stages, stream, V * P)

    copy_gbs = copy_bandwidth()
    c2 = None if a.no_c2 else c2_leg(a, dev)
    ic = None
    if not a.no_init_compare:
        full_ic = init_compare(a, ic_scenes)
        ic = {k: full_ic[k] for k in ("learned_wins", "mean_iter_ratio", "gate", "mean_psnr_gain_at", "beta_tuned",
                                      "net_final_loss", "seconds")}
        ic["iters_pca_learned"] = [[r["iters_pca"], r["iters_learned"]] for r in full_ic["tests"]]
        ic["config"] = full_ic["config"]
        print("init compare: %s" % json.dumps(full_ic), file=sys.stderr, flush=True)
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(c, pool_cams, tg, views_for_step(a.warmup + a.steps - 1))
        cpu["configs"] = cpu_baseline_configs()

    out = {
        "metric": "fwd+bwd iters/s @1.5M Gaussians, 8x720p",
        "value": round(1.0 / step_s, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "loop corridor, %d Gaussians SH3 from the voxel-PCA cascade after %d optimiser "
                               "iterations, 8 views 1280x720 per step, L1 rgb + 0.2 L1 depth, sparse Adam over 5 "
                               "latest segments" % (n, STEADY_ITERS), "gaussians": n, "views_per_step": V,
                   "width": W, "height": H, "tile": "%dx%d" % tile},
        "step_ms_p10_p50_p90": [round(float(x), 4) for x in pct],
        "iters_per_s_at_median": round(1000.0 / float(pct[1]), 3),
        "render_mode": render_mode,
        "render_modes_ms": modes,
        "at_init": at_init_out,
        "blends_per_s": round(blends / step_s, 1),
        "blends_per_step": blends,
        "instances_per_step": M,
        "visible_pairs_per_step": Nv,
        "updated_rows": Nu,
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "graph": use_graph,
        "eager_ms_per_step": round(eager_ms, 3),
        "step_alg_bytes": B_alg,
        "step_hbm_frac": round(B_alg / step_s / (HBM_PEAK_GBS * 1e9), 4),
        "step_hbm_frac_of_measured_copy": round(B_alg / step_s / (copy_gbs * 1e9), 4) if copy_gbs else None,
        "copy_GBps": round(copy_gbs, 1) if copy_gbs else None,
        "tile_autotune_s_per_step": {k: round(v, 5) for k, v in tune.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "loss_last": loss_last,
        "full_loss": full,
        "maintenance": maint,
        "loop_registration": loopr,
        "init_path": initr,
        "c2": c2,
        "learned_vs_pca_init": ic,
        "disc_map": disc,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
