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
    assert lib.gsr_abi_version() == 4


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


def test_new_entry_points_reject_invalid_arguments():
    # masks and loss, maintenance, registration, segment moves, voxel covariances: host checks only
    from paper_2604_12942_amd import _abi
    L = _abi.load()
    c = ctypes
    r = _abi.Raster(128, 96, 16, 16)
    P = c.c_void_p(1)  # never dereferenced: every call below fails validation first
    assert L.gsr_support_mask(P, 1, c.byref(r), 1.5, 2, P, P, None) == 1      # tau outside [0, 1]
    assert L.gsr_support_mask(P, 1, c.byref(r), 0.5, 9, P, P, None) == 1      # radius above 8
    assert L.gsr_loss(P, P, P, P, None, 1, c.byref(r), P, None, 1.0, 0.2, 0.2, P, P, P, P, 0, None) == 1  # mask w/o count
    assert L.gsr_loss(P, P, P, P, None, 1, c.byref(r), None, None, 1.0, 0.2, 0.2, P, P, P, P, 1, None) == 1  # ws too small
    assert L.gsr_prune_select(P, None, 0, 10, -1.0, 1.5, P, P, P, 1 << 30, None) == 1  # ratio above 1
    assert L.gsr_prune_select(P, None, 0, -1, -1.0, 0.5, P, P, P, 1 << 30, None) == 1
    g = _abi.RowGroups()
    g.n_groups = 1
    g.cols[0] = 1
    assert L.gsr_gather_rows(c.byref(g), 10, None, 5, 4, 0, None) == 1        # rows past the destination
    assert L.gsr_proximity_filter(P, 10, P, 10, 0.0, P, P, P, P, 1 << 30, None) == 1  # d_min = 0
    gs = _abi.Gaussians(None, None, None, None, None, 10, 0, 0)
    assert L.gsr_gicp_prepare(c.byref(gs), P, 0, P, 1, 30.0, 0.5, P, P, P, P, P, 1 << 30, None) == 1  # NULL means
    assert L.gsr_gicp_iterate(c.byref(gs), P, P, P, 0.5, P, P, None, -1, P, 1 << 30, None) == 1
    prm = _abi.Params(None, None, None, None, None)
    assert L.gsr_transform_segment(c.byref(prm), 10, 3, P, 0, P, P, None) == 1  # NULL parameter arrays
    assert L.gsr_transform_cameras(None, 2, None, P, None) == 1
    assert L.gsr_voxel_pca_cov(P, None, 10, 0, None, None, P, 1 << 30, None) == 1  # no point covariances
    assert L.gsr_loss_workspace(0, c.byref(r)) == 0
    # depth-sliced forward: workspace grows with the instance capacity; missing ws or a short one fails
    small, big = L.gsr_render_fwd_sliced_workspace(1, c.byref(r), 1 << 16), L.gsr_render_fwd_sliced_workspace(
        1, c.byref(r), 1 << 24)
    assert 0 < small < big and L.gsr_render_fwd_sliced_workspace(1, c.byref(r), -1) == 0
    assert L.gsr_render_fwd_sliced(P, P, P, None, P, 1, c.byref(r), P, P, P, P, 1 << 16, None, small, None) == 1
    assert L.gsr_render_fwd_sliced(P, P, P, None, P, 1, c.byref(r), P, P, P, P, 1 << 16, P, small - 1, None) == 2
    # storage order of the rows
    wo = L.gsr_row_order_workspace(1000)
    assert wo > 0 and L.gsr_row_order_workspace(-1) == 0
    assert L.gsr_row_order(None, None, 1000, P, P, wo, None) == 1          # no means
    assert L.gsr_row_order(P, None, -5, P, P, wo, None) == 1               # negative count
    assert L.gsr_row_order(P, None, 1000, P, P, wo - 1, None) == 2         # workspace too small


def test_noalloc_visible_list_rejects_sizes_beyond_its_scratch():
    # the allocation-free entry point checks n against its fixed scratch before any HIP call
    from paper_2604_12942_amd import _abi
    L = _abi.load()
    fake = ctypes.c_void_p(256)  # never dereferenced: the call is rejected on the host
    big = L.gsr_visible_list_noalloc_max() + 1
    assert L.gsr_visible_list_noalloc(fake, big, 1, fake, fake, None) == 2
    assert L.gsr_visible_list_noalloc(fake, -1, 1, fake, fake, None) == 1
    assert L.gsr_visible_list_noalloc(None, 10, 1, fake, fake, None) == 1
    assert L.gsr_visible_list_noalloc(fake, 10, 0, fake, fake, None) == 1
