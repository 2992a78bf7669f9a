"""Map maintenance around the optimisation (Sec. III-C): pruning of low-opacity Gaussians under a
bounded removal ratio, and insertion of newly initialised Gaussians after the spatial-proximity
filter against the map.  The rows of the parameters and of the per-row optimiser state (Adam
moments, segment ids) move together.  Selection, filtering and the row moves are libgsr kernels;
the host reads the surviving row count once, to size the new arrays.
"""
from __future__ import annotations

import math

import torch

from . import _abi, gather_rows, prune_select, proximity_filter, row_order


def _columns(t, rows):
    return t.numel() // rows if rows else (t.shape[0] if t.dim() > 1 else 1)


def _new_like(t, rows):
    shape = tuple(t.shape[:-1]) + (rows,)
    return torch.empty(shape, dtype=t.dtype, device=t.device)


def _gather_all(pairs, src_rows, index, n_rows, dst_rows, dst_offset):
    for s in range(0, len(pairs), _abi.MAX_ROW_GROUPS):
        gather_rows(pairs[s:s + _abi.MAX_ROW_GROUPS], src_rows, index, n_rows, dst_rows, dst_offset)


def prune(arrays, opacity_logits, min_opacity, max_ratio, segment_id=None, min_segment=0):
    """arrays: dict name -> component-major 4-byte tensor ([c, n] or [n]) to compact together
    (segment_id, when given, is compacted too if it is one of them).  Removes at most
    floor(max_ratio * n) rows with opacity below min_opacity in unfrozen segments, lowest opacity
    first.  Returns (dict of new tensors, number of removed rows)."""
    n = opacity_logits.numel()
    max_logit = math.log(min_opacity / (1.0 - min_opacity))
    keep, n_keep = prune_select(opacity_logits, max_logit, max_ratio, segment_id, min_segment)
    m = int(n_keep.item())
    out = {k: _new_like(a, m) for k, a in arrays.items()}
    _gather_all([(arrays[k], out[k]) for k in arrays], n, keep, m, m, 0)
    return out, n - m


def insert(arrays, new_arrays, d_min):
    """Appends the rows of new_arrays (same keys as arrays) whose mean lies at least d_min from
    every mean of the map ("means" [3, n]).  Returns (dict of new tensors, rows added)."""
    n = arrays["means"].shape[1]
    n_new = new_arrays["means"].shape[1]
    keep, index, n_keep = proximity_filter(arrays["means"], new_arrays["means"], d_min)
    k = int(n_keep.item())
    out = {name: _new_like(a, n + k) for name, a in arrays.items()}
    _gather_all([(arrays[name], out[name]) for name in arrays], n, None, n, n + k, 0)
    _gather_all([(new_arrays[name], out[name]) for name in arrays], n_new, index, k, n + k, n)
    return out, k


def reorder(arrays, segment_id=None):
    """Rows of arrays (same keys as for prune) moved into storage order: by segment, then by the
    Morton code of the mean (gsr_row_order).  Returns (dict of new tensors, the order)."""
    n = arrays["means"].shape[1]
    order = row_order(arrays["means"], segment_id)
    out = {k: _new_like(a, n) for k, a in arrays.items()}
    _gather_all([(arrays[k], out[k]) for k in arrays], n, order, n, n, 0)
    return out, order
