"""The allocation-free visible list (gsr_visible_list_noalloc, the library's fixed device scratch)
against the workspace entry point gsr_visible_list and against numpy, through the C ABI: two
calls in a row, the second on a smaller input, then an empty one.  Index work: bit-exact."""
import ctypes as C

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _tile_info(rng, n, V):
    ti = np.zeros((4, V * n), np.uint32)
    ti[0] = np.where(rng.random(V * n) < 0.12, rng.integers(1, 40, V * n), 0).astype(np.uint32)
    return ti


def _call(L, fn, ti, n, V, ws=None):
    dev = torch.from_numpy(ti.view(np.int32)).cuda()
    lst = torch.full((max(1, n),), -1, dtype=torch.int32, device="cuda")
    cnt = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: C.c_void_p(t.data_ptr())
    if ws is None:
        status = fn(p(dev), n, V, p(lst), p(cnt), st)
    else:
        status = fn(p(dev), n, V, p(lst), p(cnt), p(ws), ws.numel(), st)
    assert status == 0, status
    torch.cuda.synchronize()
    c = int(cnt.item())
    return c, lst[:c].cpu().numpy().astype(np.int64)


def test_noalloc_visible_list_matches_workspace_entry_point():
    from paper_2604_12942_amd import _abi
    L = _abi.load()
    rng = np.random.default_rng(20)
    assert L.gsr_visible_list_noalloc_max() == 1 << 24
    for n, V in ((1_000_003, 3), (70_001, 2), (0, 1)):
        ti = _tile_info(rng, n, V)
        print("visible list noalloc: n=%d V=%d" % (n, V), flush=True)
        ws = torch.empty(int(L.gsr_visible_list_workspace(n)), dtype=torch.uint8, device="cuda")
        c_ref, l_ref = _call(L, L.gsr_visible_list, ti, n, V, ws)
        c_got, l_got = _call(L, L.gsr_visible_list_noalloc, ti, n, V)
        exp = np.nonzero(np.any(ti[0].reshape(V, n) > 0, axis=0))[0] if n else np.zeros(0, np.int64)
        assert c_ref == len(exp) and np.array_equal(l_ref, exp)
        assert c_got == c_ref and np.array_equal(l_got, l_ref), (n, V, c_got, c_ref)
