"""The C ABI library loads and exports every entry point include/gsr.h declares (CPU only: no
compute call is made)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "gsr.h")).read()
    return sorted(set(re.findall(r"GSR_API\s+[\w\s\*]*?\b(gsr_\w+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for req in ("gsr_project", "gsr_bin_sort", "gsr_render_fwd", "gsr_render_bwd", "gsr_project_bwd",
                "gsr_adam_step", "gsr_loss_l1"):
        assert req in names


def test_library_exports_every_declared_symbol():
    from paper_2604_12942_amd import _abi
    lib = ctypes.CDLL(_abi.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    assert set(declared()) == set(_abi.EXPORTS)
    assert lib.gsr_abi_version() == 3


def test_invalid_arguments_are_rejected_before_launch():
    # argument validation happens on the host, before any HIP call
    from paper_2604_12942_amd import _abi
    L = _abi.load()
    r = _abi.Raster(128, 96, 12, 12)  # unsupported tile shape
    assert L.gsr_tiles_per_view(ctypes.byref(r)) == -1
    g = _abi.Gaussians(None, None, None, None, None, 10, 5, 0)  # sh_degree 5, NULL pointers
    r = _abi.Raster(128, 96, 16, 16)
    assert L.gsr_project(ctypes.byref(g), None, 1, ctypes.byref(r), None, None, None) == 1
    assert L.gsr_bin_sort_workspace(-1, 1, 10, ctypes.byref(r)) == 0
    assert L.gsr_status_str(1) == b"invalid argument"
