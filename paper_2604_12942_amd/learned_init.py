"""Cascaded Gaussian initialisation with the learned model branch (Sec. III-B, Eq. 3) and the
training of its per-voxel point network on maps the plain optimiser produced.

Every numerical step is a libgsr kernel (voxel PCA, point network forward / backward, cascade,
Adam); this module strings them together and keeps the buffers.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (adam_step, cascade, pointnet_backward, pointnet_forward, pointnet_weight_count,
               voxel_pca, voxel_targets)

# readings: He-uniform initial weights, Adam at 1e-3 for the network
NET_LR = 1e-3


def init_weights(seed, device="cuda"):
    """He-uniform weights and zero biases in the flat layout of gsr_pointnet_fwd."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, nout in ((3, 64), (64, 64), (64, 64), (76, 64), (64, 8)):
        lim = np.sqrt(6.0 / k)
        parts += [rng.uniform(-lim, lim, (k, nout)).ravel(), np.zeros(nout)]
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == pointnet_weight_count()
    return torch.from_numpy(w).to(device)


class SceneInit:
    """Device copies of one LiDAR-seeded scene and its voxel-PCA fit."""

    def __init__(self, points, colors, depth, segment, n_segments, seed=0, device="cuda"):
        self.n = points.shape[0]
        self.pts = torch.from_numpy(np.ascontiguousarray(points.T, np.float32)).to(device)
        self.col = torch.from_numpy(np.ascontiguousarray(colors.T, np.float32)).to(device)
        self.depth = torch.from_numpy(np.ascontiguousarray(depth, np.float32)).to(device)
        self.segment = torch.from_numpy(np.ascontiguousarray(segment, np.int32)).to(device)
        self.n_segments = int(n_segments)
        self.vox = voxel_pca(self.pts, seed)

    def gaussians(self, weights=None, beta=0.0, focal=320.0, sh_degree=3):
        """Eq. 3 cascade: the model branch where the network's prediction is valid (weights given),
        else voxel PCA where reliable, else the heuristic.  beta > 0 fixes Eq. 5's factor."""
        pred = pointnet_forward(self.pts, self.vox, weights) if weights is not None else None
        P, branch = cascade(self.pts, self.col, self.depth, self.vox, pred=pred, focal=focal, beta=beta,
                            segment=self.segment, n_segments=self.n_segments, sh_degree=sh_degree)
        return P, branch

    def targets(self, P):
        """Per-voxel training targets from optimised Gaussians seeded one per point: the mean
        covariance (xx, xy, xz, yy, yz, zz) and mean opacity over the voxel's points
        (gsr_voxel_targets)."""
        return voxel_targets(P, self.vox)


def train_pointnet(scenes, targets, weights, steps, lr=NET_LR, blocks=512, log=None):
    """Adam on the network weights; each step is one full batch over one training scene's voxels
    (round robin).  targets[k] = (cov_t, o_t, mask) of scenes[k].  Returns the mean loss of the
    last pass."""
    dev = weights.device
    nw = weights.numel()
    grad = torch.zeros(nw, dtype=torch.float32, device=dev)
    m = torch.zeros_like(weights)
    v = torch.zeros_like(weights)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    ws = None
    last = []
    for it in range(steps):
        k = it % len(scenes)
        sc = scenes[k]
        cov_t, o_t, mask = targets[k]
        cnt = max(1, int(mask.sum().item()))
        loss.zero_()
        ws = pointnet_backward(sc.pts, sc.vox, weights, cov_t, o_t, mask, 1.0 / cnt, grad, loss, blocks=blocks,
                               ws=ws)
        adam_step([(weights.view(nw, 1), grad.view(nw, 1), m.view(nw, 1), v.view(nw, 1), lr)], nw, None,
                  eps=1e-8, step=it + 1)
        if it >= steps - len(scenes):
            last.append(float(loss.item()))
        if log and (it % 50 == 0 or it == steps - 1):
            log(it, float(loss.item()))
    return float(np.mean(last)) if last else float("nan")
