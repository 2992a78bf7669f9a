"""Oracle of the map maintenance around the optimisation (Sec. III-C): low-opacity pruning under
a bounded removal ratio, and the spatial-proximity filter applied to newly initialised Gaussians
before they are inserted.  Test infrastructure only: the test-suite, the smoke check and the
benchmark's CPU baseline may use it; the product path never imports it.

Definitions (plain, no acceleration structure):

* pruning candidates: rows whose opacity logit is below max_logit (opacity below
  sigmoid(max_logit)) and that belong to an unfrozen segment (segment id >= min_segment, when
  segment ids are given).  At most k = floor(max_ratio * n) rows are removed: all candidates when
  there are at most k of them, else the k candidates with the smallest logits, equal logits in
  ascending row order.  Survivors keep their relative order.
* storage order (not a step of the method: the order in which the rows are kept, defined here so
  that the kernel's order can be checked): rows by segment id, then by the Morton code of the
  mean's cell on a 1024^3 grid over the means' bounding box (x bits lowest), then by row index.
  A coordinate's cell is floor((x - lo) * (1024 / (hi - lo))) in float32, clamped to [0, 1023].
* insertion filter: a new Gaussian is redundant when some map Gaussian's mean lies strictly
  closer than d_min.  The squared distance is evaluated in float64 from the float32 means as
  ((dx*dx + dy*dy) + dz*dz), every operation rounded separately, and compared with
  float64(d_min)^2.
"""
from __future__ import annotations

import numpy as np


def prune_select(logits, max_logit, max_ratio, segment_id=None, min_segment=0):
    """Returns (keep_index int64 ascending, removed bool [n])."""
    lg = np.asarray(logits, np.float32)
    n = lg.shape[0]
    cand = lg < np.float32(max_logit)
    if segment_id is not None:
        cand &= np.asarray(segment_id) >= min_segment
    k = int(np.floor(np.float64(np.float32(max_ratio)) * n))
    idx = np.nonzero(cand)[0]
    if idx.size > k:
        order = np.lexsort((idx, lg[idx]))  # by logit, then by row
        idx = idx[order[:k]]
    removed = np.zeros(n, bool)
    removed[idx] = True
    return np.nonzero(~removed)[0], removed


def morton_cells(means):
    """Cell of each coordinate on the 1024^3 grid over the bounding box: int64 [3, n]."""
    m = np.asarray(means, np.float32)
    out = np.zeros(m.shape, np.int64)
    for a in range(3):
        lo, hi = m[a].min(), m[a].max()
        sc = np.float32(1024) / (hi - lo) if hi > lo else np.float32(0)
        c = np.floor((m[a] - lo) * sc)
        out[a] = np.where(c >= 1023, 1023, np.maximum(c, 0)).astype(np.int64)
    return out


def morton_code(cells):
    """Interleave the ten bits of the x, y and z cells, bit b of axis a at 3b + a."""
    q = np.asarray(cells, np.int64)
    code = np.zeros(q.shape[1:], np.int64)
    for b in range(10):
        for a in range(3):
            code |= ((q[a] >> b) & 1) << (3 * b + a)
    return code


def row_order(means, segment_id=None):
    """The storage order: position j holds the row order[j] (int64)."""
    n = np.asarray(means).shape[1]
    code = morton_code(morton_cells(means))
    seg = np.zeros(n, np.int64) if segment_id is None else np.asarray(segment_id, np.int64)
    return np.lexsort((np.arange(n), code, seg))


def gather_rows(arr, index):
    """Component-major [c, n] (or [n]) rows picked by index."""
    a = np.asarray(arr)
    return a[..., np.asarray(index)]


def redundant(map_means, new_means, d_min, chunk=2048):
    """bool [M]: new mean j has a map mean strictly within d_min (float64 test, see above)."""
    A = np.asarray(map_means, np.float32).astype(np.float64)   # [3, N]
    B = np.asarray(new_means, np.float32).astype(np.float64)   # [3, M]
    dd = np.float64(np.float32(d_min)) * np.float64(np.float32(d_min))
    M = B.shape[1]
    out = np.zeros(M, bool)
    if A.shape[1] == 0:
        return out
    for s in range(0, M, chunk):
        b = B[:, s:s + chunk]
        dx = b[0][:, None] - A[0][None, :]
        dy = b[1][:, None] - A[1][None, :]
        dz = b[2][:, None] - A[2][None, :]
        d2 = (dx * dx + dy * dy) + dz * dz
        out[s:s + chunk] = np.any(d2 < dd, axis=1)
    return out
