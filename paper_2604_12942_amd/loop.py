"""Gaussian-based loop closure (Sec. III-D): registration of a loopframe's Gaussians against the
map Gaussians seen from the views around a historical loopframe (Eq. 13-16), with the
acceptance test, and propagation of a corrected pose to a segment of the map.

Registration runs on the device end to end (set extraction, covariances, grid, Gauss-Newton with
an on-device 6x6 solve); the host reads the statistics once, after the queued iterations.
"""
from __future__ import annotations

import numpy as np
import torch

from . import gicp_iterate, gicp_prepare

# readings: correspondences within 0.5 m; queries limited to 30 m from a keyframe centre;
# accepted when converged with at least 100 correspondences and mean r^T W r below 1
D_CORR, D_MAX = 0.5, 30.0
MIN_CORR, ACCEPT_COST = 100, 1.0


def register(P, sh_degree, segment_id, src_segment, cams, n_cams, pose0=None, d_max=D_MAX, d_corr=D_CORR,
             max_iter=30, state=None):
    """Aligns the Gaussians of segment src_segment to the target set seen from cams (device
    gsr_camera records).  pose0: (R [3, 3], t [3]) initial guess (identity by default).
    Returns a dict with R, t, converged, failed, iterations, count, cost, rmse, accepted, state."""
    dev = P["means"].device
    state = gicp_prepare(P, sh_degree, segment_id, src_segment, cams, n_cams, d_max, d_corr, state)
    R0, t0 = (np.eye(3), np.zeros(3)) if pose0 is None else pose0
    pose = torch.tensor(np.concatenate([np.asarray(R0, np.float64).ravel(), np.asarray(t0, np.float64)]),
                        dtype=torch.float64, device=dev)
    gicp_iterate(P, sh_degree, state, pose, max_iter)
    st = state["stats"].cpu().numpy()
    pz = pose.cpu().numpy()
    count = int(st[29])
    conv, failed = bool(st[36]), bool(st[38])
    cost = float(st[27])
    accepted = conv and not failed and count >= MIN_CORR and cost / count < ACCEPT_COST
    return dict(R=pz[:9].reshape(3, 3), t=pz[9:], converged=conv, failed=failed, iterations=int(st[37]),
                count=count, cost=cost, rmse=float(np.sqrt(st[28] / max(count, 1))), accepted=accepted,
                n_src=int(state["counts"][0].item()), n_tgt=int(state["counts"][1].item()), state=state)
