"""ctypes declarations of include/gsr.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsr.so")

P = C.c_void_p


class Camera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("z_near", C.c_float), ("bg", C.c_float * 3),
                ("width", C.c_int32), ("height", C.c_int32), ("_pad", C.c_int32 * 2)]


class Gaussians(C.Structure):
    _fields_ = [("means", P), ("log_scales", P), ("quats", P), ("opacity_logits", P), ("sh", P),
                ("n", C.c_int64), ("sh_degree", C.c_int32), ("_pad", C.c_int32)]


class ParamGrads(C.Structure):
    _fields_ = [("means", P), ("log_scales", P), ("quats", P), ("opacity_logits", P), ("sh", P)]


class Raster(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32)]


class AdamFused(C.Structure):
    _fields_ = [("m", ParamGrads), ("v", ParamGrads), ("lr", C.c_float * 6), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("step", P)]


MAX_GROUPS = 8


class AdamGroups(C.Structure):
    _fields_ = [("param", P * MAX_GROUPS), ("grad", P * MAX_GROUPS), ("m", P * MAX_GROUPS), ("v", P * MAX_GROUPS),
                ("cols", C.c_int32 * MAX_GROUPS), ("lr", C.c_float * MAX_GROUPS), ("n_groups", C.c_int32),
                ("_pad", C.c_int32)]


class Emission(C.Structure):
    _fields_ = [("inst_emit", C.c_void_p), ("pair_gid", C.c_void_p), ("pair_first", C.c_void_p),
                ("n_pairs", C.c_void_p)]


class Voxels(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("n_voxels", "n_outside", "key", "start", "count", "point_order",
                                          "point_voxel", "mu", "evals", "R", "s_pca", "trace", "cls", "reliable")]


MAX_ROW_GROUPS = 16


class RowGroups(C.Structure):
    _fields_ = [("src", P * MAX_ROW_GROUPS), ("dst", P * MAX_ROW_GROUPS), ("cols", C.c_int32 * MAX_ROW_GROUPS),
                ("n_groups", C.c_int32), ("_pad", C.c_int32)]


class Params(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("means", "log_scales", "quats", "opacity_logits", "sh")]


assert C.sizeof(Camera) == 96
CAMERA_BYTES = C.sizeof(Camera)
assert C.sizeof(Gaussians) == 56

SPLAT_BYTES = 48
SPLAT_GRAD_FLOATS = 10

_SIGS = {
    "gsr_abi_version": ([], C.c_int),
    "gsr_status_str": ([C.c_int], C.c_char_p),
    "gsr_tiles_per_view": ([C.POINTER(Raster)], C.c_int64),
    "gsr_project": ([C.POINTER(Gaussians), P, C.c_int32, C.POINTER(Raster), P, P, P], C.c_int),
    "gsr_bin_sort_workspace": ([C.c_int64, C.c_int32, C.c_int64, C.POINTER(Raster)], C.c_size_t),
    "gsr_bin_sort": ([P, C.c_int64, C.c_int32, C.POINTER(Raster), P, C.POINTER(Emission), C.c_int64, P, P, P, P,
                      C.c_size_t, P], C.c_int),
    "gsr_render_fwd": ([P, P, P, P, P, C.c_int32, C.POINTER(Raster), P, P, P, P, P, P], C.c_int),
    "gsr_render_bwd": ([P, P, P, P, P, P, C.c_int32, C.POINTER(Raster), P, P, P, P, P, P, C.c_size_t, C.c_int64, P],
                       C.c_int),
    "gsr_render_fwd_sliced_workspace": ([C.c_int32, C.POINTER(Raster), C.c_int64], C.c_size_t),
    "gsr_render_fwd_sliced": ([P, P, P, P, P, C.c_int32, C.POINTER(Raster), P, P, P, P, C.c_int64, P, C.c_size_t, P],
                              C.c_int),
    "gsr_render_fwd_stored_workspace": ([C.c_int32, C.POINTER(Raster)], C.c_size_t),
    "gsr_render_fwd_stored": ([P, P, P, P, P, C.c_int32, C.POINTER(Raster), P, P, P, P, P, P, P, C.c_int64, P, P,
                               C.c_size_t, P], C.c_int),
    "gsr_render_bwd_stored": ([P, P, P, P, P, P, C.c_int32, C.POINTER(Raster), P, P, P, P, C.c_int64, P, P, P, P],
                              C.c_int),
    "gsr_pair_grads": ([P, C.POINTER(Emission), P, C.c_int64, C.c_int32, P, P], C.c_int),
    "gsr_render_bwd_l1_workspace": ([C.c_int32, C.POINTER(Raster)], C.c_size_t),
    "gsr_render_bwd_l1": ([P, P, P, P, P, P, C.c_int32, C.POINTER(Raster), P, P, P, P, P, P, P, C.c_float, P, P, P,
                           C.c_size_t, P, C.c_size_t, C.c_int64, P], C.c_int),
    "gsr_render_step_workspace": ([C.c_int32, C.POINTER(Raster), C.c_int64], C.c_size_t),
    "gsr_render_step": ([P, P, P, P, P, P, C.c_int32, C.POINTER(Raster), P, P, P, C.c_float, P, P, P, P, P, P,
                         C.c_int64, P, C.c_size_t, P], C.c_int),
    "gsr_project_bwd_workspace": ([C.c_int64, C.c_int32], C.c_size_t),
    "gsr_project_bwd": ([C.POINTER(Gaussians), P, C.c_int32, C.POINTER(Raster), P, P, C.POINTER(Emission), P,
                         C.POINTER(ParamGrads), P, P, C.c_int32, P, P, C.c_size_t, P], C.c_int),
    "gsr_project_bwd_adam": ([C.POINTER(Gaussians), P, C.c_int32, C.POINTER(Raster), P, P, C.POINTER(Emission), P,
                              P, P, P, C.c_int32, C.POINTER(AdamFused), P, P, P, C.c_size_t, P], C.c_int),
    "gsr_visible_list_workspace": ([C.c_int64], C.c_size_t),
    "gsr_visible_list": ([P, C.c_int64, C.c_int32, P, P, P, C.c_size_t, P], C.c_int),
    "gsr_visible_list_noalloc_max": ([], C.c_int64),
    "gsr_visible_list_noalloc": ([P, C.c_int64, C.c_int32, P, P, P], C.c_int),
    "gsr_adam_step": ([C.POINTER(AdamGroups), C.c_int64, P, C.c_float, C.c_float, C.c_float, C.c_int32, P], C.c_int),
    "gsr_step_prep": ([P, C.c_int32, P, C.c_int32, P, P, P, P, P, C.c_int64, P], C.c_int),
    "gsr_loss_l1": ([P, P, P, P, P, C.c_int32, C.POINTER(Raster), C.c_float, P, P, P, P], C.c_int),
    "gsr_fill_u32": ([P, C.c_uint32, C.c_int64, P], C.c_int),
    "gsr_support_mask": ([P, C.c_int32, C.POINTER(Raster), C.c_float, C.c_int32, P, P, P], C.c_int),
    "gsr_loss_workspace": ([C.c_int32, C.POINTER(Raster)], C.c_size_t),
    "gsr_transform_segment": ([C.POINTER(Params), C.c_int64, C.c_int32, P, C.c_int32, P, P, P], C.c_int),
    "gsr_transform_cameras": ([P, C.c_int32, P, P, P], C.c_int),
    "gsr_gicp_workspace": ([C.c_int64], C.c_size_t),
    "gsr_gicp_prepare": ([C.POINTER(Gaussians), P, C.c_int32, P, C.c_int32, C.c_float, C.c_float, P, P, P, P, P,
                          C.c_size_t, P], C.c_int),
    "gsr_gicp_iterate": ([C.POINTER(Gaussians), P, P, P, C.c_float, P, P, P, C.c_int32, P, C.c_size_t, P], C.c_int),
    "gsr_prune_workspace": ([C.c_int64], C.c_size_t),
    "gsr_row_order_workspace": ([C.c_int64], C.c_size_t),
    "gsr_row_order": ([P, P, C.c_int64, P, P, C.c_size_t, P], C.c_int),
    "gsr_prune_select": ([P, P, C.c_int32, C.c_int64, C.c_float, C.c_float, P, P, P, C.c_size_t, P], C.c_int),
    "gsr_gather_rows": ([C.POINTER(RowGroups), C.c_int64, P, C.c_int64, C.c_int64, C.c_int64, P], C.c_int),
    "gsr_proximity_workspace": ([C.c_int64, C.c_int64], C.c_size_t),
    "gsr_proximity_filter": ([P, C.c_int64, P, C.c_int64, C.c_float, P, P, P, P, C.c_size_t, P], C.c_int),
    "gsr_loss": ([P, P, P, P, P, C.c_int32, C.POINTER(Raster), P, P, C.c_float, C.c_float, C.c_float, P, P, P, P,
                  C.c_size_t, P], C.c_int),
    "gsr_voxel_pca_workspace": ([C.c_int64], C.c_size_t),
    "gsr_voxel_pca": ([P, C.c_int64, C.c_uint64, C.POINTER(Voxels), P, C.c_size_t, P], C.c_int),
    "gsr_voxel_pca_cov": ([P, P, C.c_int64, C.c_uint64, C.POINTER(Voxels), P, P, C.c_size_t, P], C.c_int),
    "gsr_voxel_targets": ([C.POINTER(Params), C.c_int64, C.POINTER(Voxels), P, P, P, P], C.c_int),
    "gsr_pointnet_weight_count": ([], C.c_int),
    "gsr_pointnet_fwd": ([P, C.c_int64, C.POINTER(Voxels), P, P, P], C.c_int),
    "gsr_pointnet_bwd_workspace": ([C.c_int32], C.c_size_t),
    "gsr_pointnet_bwd": ([P, C.c_int64, C.POINTER(Voxels), P, P, P, P, C.c_float, C.c_int32, P, P, P, C.c_size_t,
                          P], C.c_int),
    "gsr_cascade_workspace": ([C.c_int32], C.c_size_t),
    "gsr_cascade": ([P, P, P, P, C.c_int32, C.c_int64, C.POINTER(Voxels), P, C.c_float, C.c_float, C.c_int32,
                     C.POINTER(Params), P, P, C.c_size_t, P], C.c_int),
    "gsr_cascade_anchored": ([P, P, P, P, C.c_int32, C.c_int64, C.POINTER(Voxels), P, C.c_float, C.c_float,
                              C.c_int32, C.POINTER(Params), P, P, C.c_size_t, P], C.c_int),
}

EXPORTS = tuple(_SIGS)

_lib = None


def load():
    """Load libgsr.so; fail loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgsr.so is not built: run __graft_entry__.build() (hipcc for gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


class GsrError(RuntimeError):
    pass


def check(status, what):
    if status != 0:
        raise GsrError("%s failed: %s (status %d)" % (what, load().gsr_status_str(status).decode(), status))
