// C ABI entry points: argument validation, then launches on the caller's stream.
#include "gsr_internal.h"
#include <cmath>

using namespace gsr;

extern "C" gsr_status gsr_project_launch(const gsr_gaussians *, const gsr_camera *, int, const gsr_raster *,
                                         gsr_splat *, uint32_t *, hipStream_t);
extern "C" gsr_status gsr_project_bwd_launch(const gsr_gaussians *, const gsr_camera *, int, const gsr_raster *,
                                             const gsr_splat *, const float *, const gsr_emission *,
                                             const gsr_param_grads *, double *, const uint32_t *, const int32_t *,
                                             int32_t, uint8_t *, const gsr_adam_fused *, const uint32_t *,
                                             const uint32_t *, void *, hipStream_t);
extern "C" size_t gsr_visible_list_ws_bytes(int64_t n);
extern "C" gsr_status gsr_visible_list_launch(const uint32_t *, int64_t, int, uint32_t *, uint32_t *, void *,
                                              hipStream_t);
extern "C" size_t gsr_bin_sort_ws_bytes(int64_t VN, int64_t cap, int64_t VT);
extern "C" gsr_status gsr_bin_sort_launch(uint32_t *, int64_t, int, int, int, uint32_t *, const gsr_emission *,
                                          int64_t, uint32_t *, uint32_t *, uint32_t *, void *, hipStream_t);
extern "C" size_t gsr_render_fwd_ws_bytes(int, const gsr_raster *, int64_t);
extern "C" gsr_status gsr_render_fwd_launch(const gsr_splat *, const uint32_t *, const uint32_t *, const uint32_t *,
                                            const gsr_camera *, int, const gsr_raster *, float *, float *, float *,
                                            uint32_t *, uint32_t *, int64_t, void *, hipStream_t);
extern "C" size_t gsr_render_bwd_l1_ws_bytes(int, const gsr_raster *);
extern "C" gsr_status gsr_render_bwd_l1_launch(const gsr_splat *, const uint32_t *, const uint32_t *, const uint32_t *,
                                               const uint32_t *, const gsr_camera *, int, const gsr_raster *,
                                               const float *, const float *, const float *, const uint32_t *,
                                               const float *, const float *, const int32_t *, float, double *, float *,
                                               void *, void *, int64_t, hipStream_t);
extern "C" size_t gsr_render_step_ws_bytes(int, const gsr_raster *, int64_t);
extern "C" gsr_status gsr_render_step_launch(const gsr_splat *, const uint32_t *, const uint32_t *, const uint32_t *,
                                             const uint32_t *, const gsr_camera *, int, const gsr_raster *,
                                             const float *, const float *, const int32_t *, float, float *, float *,
                                             float *, uint32_t *, double *, float *, int64_t, void *, hipStream_t);
extern "C" gsr_status gsr_render_bwd_launch(const gsr_splat *, const uint32_t *, const uint32_t *, const uint32_t *,
                                            const uint32_t *, const gsr_camera *, int, const gsr_raster *, const float *,
                                            const uint32_t *, const float *, const float *, float *, void *, int64_t,
                                            hipStream_t);
extern "C" gsr_status gsr_pair_grads_launch(const float *, const gsr_emission *, const uint32_t *, int64_t, float *,
                                            bool, hipStream_t);
extern "C" gsr_status gsr_render_store_launch(const gsr_splat *, const uint32_t *, const uint32_t *, const uint32_t *,
                                             const gsr_camera *, int, const gsr_raster *, const uint32_t *, uint32_t *,
                                             uint32_t, hipStream_t);
extern "C" gsr_status gsr_render_bwd_stored_launch(const gsr_splat *, const uint32_t *, const uint32_t *,
                                                   const uint32_t *, const uint32_t *, const gsr_camera *, int,
                                                   const gsr_raster *, const float *, const uint32_t *,
                                                   const uint32_t *, const uint32_t *, uint32_t, const float *,
                                                   const float *, float *, hipStream_t);
extern "C" size_t gsr_scan_ws_bytes(int64_t n);
extern "C" size_t gsr_row_order_ws_bytes(int64_t n);
extern "C" gsr_status gsr_row_order_launch(const float *, const int32_t *, int64_t, uint32_t *, void *, hipStream_t);
extern "C" gsr_status gsr_scan_launch(const uint32_t *, int64_t, uint32_t *, uint32_t *, void *, hipStream_t);
extern "C" size_t gsr_voxel_pca_ws_bytes(int64_t n);
extern "C" gsr_status gsr_voxel_pca_launch(const float *, int64_t, uint64_t, const gsr_voxels *, void *, hipStream_t);
extern "C" gsr_status gsr_voxel_pca_cov_launch(const float *, const float *, int64_t, uint64_t, const gsr_voxels *,
                                               float *, void *, hipStream_t);
extern "C" size_t gsr_cascade_ws_bytes(int nseg);
extern "C" gsr_status gsr_cascade_launch(const float *, const float *, const float *, const int32_t *, int, int64_t,
                                         const gsr_voxels *, const float *, float, float, int, const gsr_params *,
                                         uint8_t *, void *, hipStream_t, int);
extern "C" gsr_status gsr_voxel_targets_launch(const gsr_params *, int64_t, const gsr_voxels *, float *, float *,
                                              uint8_t *, hipStream_t);
extern "C" int gsr_pointnet_weight_count(void);
extern "C" gsr_status gsr_pointnet_fwd_launch(const float *, int64_t, const gsr_voxels *, const float *, float *,
                                              hipStream_t);
extern "C" size_t gsr_pointnet_bwd_ws_bytes(int blocks);
extern "C" gsr_status gsr_pointnet_bwd_launch(const float *, int64_t, const gsr_voxels *, const float *, const float *,
                                              const float *, const uint8_t *, float, int, float *, double *, void *,
                                              hipStream_t);
extern "C" gsr_status gsr_adam_launch(const gsr_adam_groups *, int64_t, const uint8_t *, float, float, float, int,
                                      hipStream_t);
extern "C" gsr_status gsr_loss_l1_launch(const float *, const float *, const float *, const float *, const int32_t *,
                                         int, const gsr_raster *, float, double *, float *, float *, hipStream_t);
extern "C" gsr_status gsr_fill_u32_launch(void *, uint32_t, int64_t, hipStream_t);
extern "C" gsr_status gsr_transform_segment_launch(const gsr_params *, int64_t, int, const int32_t *, int32_t,
                                                   const double *, double *, hipStream_t);
extern "C" gsr_status gsr_transform_cameras_launch(gsr_camera *, int, const uint8_t *, const double *, hipStream_t);
extern "C" size_t gsr_gicp_ws_bytes(int64_t);
extern "C" gsr_status gsr_gicp_prepare_launch(const gsr_gaussians *, const int32_t *, int32_t, const gsr_camera *, int,
                                              float, float, uint32_t *, uint32_t *, uint32_t *, double *, void *,
                                              hipStream_t);
extern "C" gsr_status gsr_gicp_iterate_launch(const gsr_gaussians *, const uint32_t *, const uint32_t *,
                                              const uint32_t *, float, double *, double *, int32_t *, int, void *,
                                              hipStream_t);
extern "C" size_t gsr_prune_ws_bytes(int64_t);
extern "C" gsr_status gsr_prune_launch(const float *, const int32_t *, int32_t, int64_t, float, uint64_t, uint32_t *,
                                       uint32_t *, void *, hipStream_t);
extern "C" gsr_status gsr_gather_launch(const gsr_row_groups *, int64_t, const uint32_t *, int64_t, int64_t, int64_t,
                                        hipStream_t);
extern "C" size_t gsr_proximity_ws_bytes(int64_t, int64_t);
extern "C" gsr_status gsr_proximity_launch(const float *, int64_t, const float *, int64_t, float, uint8_t *, uint32_t *,
                                           uint32_t *, void *, hipStream_t);
extern "C" size_t gsr_loss_ws_bytes(int, const gsr_raster *);
extern "C" gsr_status gsr_support_mask_launch(const float *, int, const gsr_raster *, float, int, uint8_t *, uint32_t *,
                                              hipStream_t);
extern "C" gsr_status gsr_loss_launch(const float *, const float *, const float *, const float *, const int32_t *, int,
                                      const gsr_raster *, const uint8_t *, const uint32_t *, float, float, float,
                                      double *, float *, float *, void *, hipStream_t);
extern "C" gsr_status gsr_tile_order_identity(uint32_t *, int64_t, hipStream_t);

namespace {

bool raster_ok(const gsr_raster *r) {
    return r && r->width > 0 && r->height > 0 && r->width <= 65535 * 8 && r->height <= 65535 * 8 &&
           valid_tile(r->tile_w, r->tile_h);
}

bool gauss_ok(const gsr_gaussians *g) {
    if (!g || g->n < 0 || g->sh_degree < 0 || g->sh_degree > 3) return false;
    if (g->n == 0) return true;
    return g->means && g->log_scales && g->quats && g->opacity_logits && g->sh;
}

int64_t tiles(const gsr_raster *r) {
    return ceil_div(r->width, r->tile_w) * ceil_div(r->height, r->tile_h);
}

hipStream_t S(gsr_stream s) { return static_cast<hipStream_t>(s); }

int64_t pixels(int32_t V, const gsr_raster *r) { return (int64_t)V * r->width * r->height; }

bool emission_ok(const gsr_emission *em) { return em && em->pair_gid && em->pair_first && em->n_pairs; }

}  // namespace

extern "C" int gsr_abi_version(void) { return GSR_ABI_VERSION; }

extern "C" const char *gsr_status_str(int status) {
    switch (status) {
        case GSR_OK: return "ok";
        case GSR_E_INVALID: return "invalid argument";
        case GSR_E_CAPACITY: return "workspace too small";
        case GSR_E_HIP: return "HIP launch or runtime error";
        case GSR_E_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

extern "C" int64_t gsr_tiles_per_view(const gsr_raster *r) { return raster_ok(r) ? tiles(r) : -1; }

extern "C" gsr_status gsr_project(const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                  const gsr_raster *r, gsr_splat *splats, uint32_t *tile_info, gsr_stream stream) {
    if (!gauss_ok(g) || !raster_ok(r) || n_views < 1 || !cams) return GSR_E_INVALID;
    if ((int64_t)n_views * g->n >= (int64_t)UINT32_MAX) return GSR_E_INVALID;
    if (g->n > 0 && (!splats || !tile_info)) return GSR_E_INVALID;
    if (ceil_div(r->width, r->tile_w) > 65535 || ceil_div(r->height, r->tile_h) > 65535) return GSR_E_UNSUPPORTED;
    return gsr_project_launch(g, cams, n_views, r, splats, tile_info, S(stream));
}

extern "C" size_t gsr_bin_sort_workspace(int64_t n, int32_t n_views, int64_t capacity, const gsr_raster *r) {
    if (n < 0 || n_views < 1 || capacity < 0 || !raster_ok(r)) return 0;
    return gsr_bin_sort_ws_bytes((int64_t)n_views * n, capacity, (int64_t)n_views * tiles(r));
}

extern "C" gsr_status gsr_bin_sort(uint32_t *tile_info, int64_t n, int32_t n_views, const gsr_raster *r,
                                   uint32_t *inst_gid, const gsr_emission *em, int64_t capacity,
                                   uint32_t *tile_ranges, uint32_t *n_instances, uint32_t *tile_order, void *ws,
                                   size_t ws_bytes, gsr_stream stream) {
    if (!raster_ok(r) || n < 0 || n_views < 1 || capacity < 1 || capacity >= (int64_t)UINT32_MAX) return GSR_E_INVALID;
    if ((int64_t)n_views * n >= (int64_t)UINT32_MAX) return GSR_E_INVALID;
    if (!tile_info && n > 0) return GSR_E_INVALID;
    if (!inst_gid || !tile_ranges || !n_instances || !ws) return GSR_E_INVALID;
    if (em && (!em->inst_emit || !em->pair_gid || !em->pair_first || !em->n_pairs)) return GSR_E_INVALID;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return GSR_E_INVALID;
    if (ws_bytes < gsr_bin_sort_ws_bytes((int64_t)n_views * n, capacity, (int64_t)n_views * tiles(r)))
        return GSR_E_CAPACITY;
    if ((int64_t)n_views * tiles(r) > (int64_t)(1u << 24)) return GSR_E_UNSUPPORTED;
    const int ntx = (int)ceil_div(r->width, r->tile_w), nty = (int)ceil_div(r->height, r->tile_h);
    if (n == 0) {
        gsr_status s = gsr_fill_u32_launch(tile_ranges, 0u, 2 * (int64_t)n_views * ntx * nty, S(stream));
        if (s != GSR_OK) return s;
        if (tile_order) {
            // no instances: any order of the view-tiles; identity
            s = gsr_tile_order_identity(tile_order, (int64_t)n_views * ntx * nty, S(stream));
            if (s != GSR_OK) return s;
        }
        if (em) {
            s = gsr_fill_u32_launch(em->n_pairs, 0u, 1, S(stream));
            if (s != GSR_OK) return s;
        }
        return gsr_fill_u32_launch(n_instances, 0u, 1, S(stream));
    }
    return gsr_bin_sort_launch(tile_info, n, n_views, ntx, nty, inst_gid, em, capacity, tile_ranges, n_instances,
                               tile_order, ws, S(stream));
}

extern "C" gsr_status gsr_render_fwd(const gsr_splat *splats, const uint32_t *inst_gid, const uint32_t *tile_ranges,
                                     const uint32_t *tile_order, const gsr_camera *cams, int32_t n_views, const gsr_raster *r, float *rgb,
                                     float *depth, float *T_final, uint32_t *last, uint32_t *n_contrib,
                                     gsr_stream stream) {
    if (!raster_ok(r) || n_views < 1 || !cams || !tile_ranges || !rgb || !depth || !T_final || !last)
        return GSR_E_INVALID;
    return gsr_render_fwd_launch(splats, inst_gid, tile_ranges, tile_order, cams, n_views, r, rgb, depth, T_final,
                                 last, n_contrib, 0, nullptr, S(stream));
}

extern "C" size_t gsr_render_fwd_sliced_workspace(int32_t n_views, const gsr_raster *r, int64_t capacity) {
    if (!raster_ok(r) || n_views < 1 || capacity < 0) return 0;
    return gsr_render_fwd_ws_bytes(n_views, r, capacity);
}

extern "C" gsr_status gsr_render_fwd_sliced(const gsr_splat *splats, const uint32_t *inst_gid,
                                            const uint32_t *tile_ranges, const uint32_t *tile_order,
                                            const gsr_camera *cams, int32_t n_views, const gsr_raster *r, float *rgb,
                                            float *depth, float *T_final, uint32_t *last, int64_t capacity, void *ws,
                                            size_t ws_bytes, gsr_stream stream) {
    if (!raster_ok(r) || n_views < 1 || !cams || !tile_ranges || !rgb || !depth || !T_final || !last || !ws ||
        capacity < 0 || capacity >= (int64_t)UINT32_MAX)
        return GSR_E_INVALID;
    if (ws_bytes < gsr_render_fwd_ws_bytes(n_views, r, capacity)) return GSR_E_CAPACITY;
    return gsr_render_fwd_launch(splats, inst_gid, tile_ranges, tile_order, cams, n_views, r, rgb, depth, T_final,
                                 last, nullptr, capacity, ws, S(stream));
}

extern "C" gsr_status gsr_render_bwd(const gsr_splat *splats, const uint32_t *inst_gid, const uint32_t *inst_emit,
                                     const uint32_t *tile_ranges, const uint32_t *tile_order, const gsr_camera *cams,
                                     int32_t n_views, const gsr_raster *r, const float *T_final, const uint32_t *last,
                                     const float *dL_drgb, const float *dL_ddepth, float *dinst, void *fwd_ws,
                                     size_t fwd_ws_bytes, int64_t capacity, gsr_stream stream) {
    if (!raster_ok(r) || n_views < 1 || !cams || !tile_ranges || !T_final || !last || !dL_drgb || !dinst ||
        !inst_emit || !inst_gid || !splats)
        return GSR_E_INVALID;
    if (fwd_ws) {
        if (capacity < 0 || capacity >= (int64_t)UINT32_MAX || (reinterpret_cast<uintptr_t>(fwd_ws) & 255) != 0)
            return GSR_E_INVALID;
        if (fwd_ws_bytes < gsr_render_fwd_ws_bytes(n_views, r, capacity)) return GSR_E_CAPACITY;
    }
    return gsr_render_bwd_launch(splats, inst_gid, inst_emit, tile_ranges, tile_order, cams, n_views, r, T_final, last,
                                 dL_drgb, dL_ddepth, dinst, fwd_ws, capacity, S(stream));
}

extern "C" size_t gsr_render_bwd_l1_workspace(int32_t n_views, const gsr_raster *r) {
    if (!raster_ok(r) || n_views < 1) return 0;
    return gsr_render_bwd_l1_ws_bytes(n_views, r);
}

extern "C" gsr_status gsr_render_bwd_l1(const gsr_splat *splats, const uint32_t *inst_gid, const uint32_t *inst_emit,
                                        const uint32_t *tile_ranges, const uint32_t *tile_order,
                                        const gsr_camera *cams, int32_t n_views, const gsr_raster *r, const float *rgb,
                                        const float *depth, const float *T_final, const uint32_t *last,
                                        const float *target_rgb, const float *target_depth,
                                        const int32_t *target_index, float lambda_depth, double *loss, float *dinst,
                                        void *ws, size_t ws_bytes, void *fwd_ws, size_t fwd_ws_bytes,
                                        int64_t capacity, gsr_stream stream) {
    if (!raster_ok(r) || n_views < 1) return GSR_E_INVALID;
    if (!splats || !inst_gid || !inst_emit || !tile_ranges || !cams || !rgb || !depth || !T_final || !last ||
        !target_rgb || !loss || !dinst || !ws)
        return GSR_E_INVALID;
    if (!(lambda_depth >= 0.f)) return GSR_E_INVALID;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return GSR_E_INVALID;
    if (ws_bytes < gsr_render_bwd_l1_ws_bytes(n_views, r)) return GSR_E_CAPACITY;
    if (fwd_ws) {
        if (capacity < 0 || capacity >= (int64_t)UINT32_MAX || (reinterpret_cast<uintptr_t>(fwd_ws) & 255) != 0)
            return GSR_E_INVALID;
        if (fwd_ws_bytes < gsr_render_fwd_ws_bytes(n_views, r, capacity)) return GSR_E_CAPACITY;
    }
    return gsr_render_bwd_l1_launch(splats, inst_gid, inst_emit, tile_ranges, tile_order, cams, n_views, r, rgb, depth,
                                    T_final, last, target_rgb, target_depth, target_index, lambda_depth, loss, dinst,
                                    ws, fwd_ws, capacity, S(stream));
}

extern "C" size_t gsr_render_step_workspace(int32_t n_views, const gsr_raster *r, int64_t capacity) {
    if (!raster_ok(r) || n_views < 1 || capacity < 1) return 0;
    return gsr_render_step_ws_bytes(n_views, r, capacity);
}

extern "C" gsr_status gsr_render_step(const gsr_splat *splats, const uint32_t *inst_gid, const uint32_t *inst_emit,
                                      const uint32_t *tile_ranges, const uint32_t *tile_order, const gsr_camera *cams,
                                      int32_t n_views, const gsr_raster *r, const float *target_rgb,
                                      const float *target_depth, const int32_t *target_index, float lambda_depth,
                                      float *rgb, float *depth, float *T_final, uint32_t *last, double *loss,
                                      float *dinst, int64_t capacity, void *ws, size_t ws_bytes, gsr_stream stream) {
    if (!raster_ok(r) || n_views < 1 || capacity < 1 || capacity >= (int64_t)UINT32_MAX) return GSR_E_INVALID;
    if (!splats || !inst_gid || !inst_emit || !tile_ranges || !cams || !target_rgb || !rgb || !depth || !T_final ||
        !last || !loss || !dinst || !ws)
        return GSR_E_INVALID;
    if (!(lambda_depth >= 0.f)) return GSR_E_INVALID;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return GSR_E_INVALID;
    if (ws_bytes < gsr_render_step_ws_bytes(n_views, r, capacity)) return GSR_E_CAPACITY;
    return gsr_render_step_launch(splats, inst_gid, inst_emit, tile_ranges, tile_order, cams, n_views, r, target_rgb,
                                  target_depth, target_index, lambda_depth, rgb, depth, T_final, last, loss, dinst,
                                  capacity, ws, S(stream));
}

extern "C" size_t gsr_render_fwd_stored_workspace(int32_t n_views, const gsr_raster *r) {
    if (!raster_ok(r) || n_views < 1) return 0;
    return gsr_scan_ws_bytes(pixels(n_views, r));
}

extern "C" gsr_status gsr_render_fwd_stored(const gsr_splat *splats, const uint32_t *inst_gid,
                                            const uint32_t *tile_ranges, const uint32_t *tile_order,
                                            const gsr_camera *cams, int32_t n_views, const gsr_raster *r, float *rgb,
                                            float *depth, float *T_final, uint32_t *last, uint32_t *n_contrib,
                                            uint32_t *contrib_offsets, uint32_t *contrib_ids,
                                            int64_t contrib_capacity, uint32_t *n_contrib_total, void *ws,
                                            size_t ws_bytes, gsr_stream stream) {
    if (!raster_ok(r) || n_views < 1 || !cams || !tile_ranges || !rgb || !depth || !T_final || !last || !n_contrib ||
        !contrib_offsets || !contrib_ids || !n_contrib_total || !ws || !splats || !inst_gid)
        return GSR_E_INVALID;
    if (contrib_capacity < 1 || contrib_capacity >= (int64_t)UINT32_MAX) return GSR_E_INVALID;
    if (ws_bytes < gsr_render_fwd_stored_workspace(n_views, r)) return GSR_E_CAPACITY;
    gsr_status s = gsr_render_fwd_launch(splats, inst_gid, tile_ranges, tile_order, cams, n_views, r, rgb, depth,
                                         T_final, last, n_contrib, 0, nullptr, S(stream));
    if (s != GSR_OK) return s;
    s = gsr_scan_launch(n_contrib, pixels(n_views, r), contrib_offsets, n_contrib_total, ws, S(stream));
    if (s != GSR_OK) return s;
    return gsr_render_store_launch(splats, inst_gid, tile_ranges, tile_order, cams, n_views, r, contrib_offsets,
                                   contrib_ids, (uint32_t)contrib_capacity, S(stream));
}

extern "C" gsr_status gsr_render_bwd_stored(const gsr_splat *splats, const uint32_t *inst_gid,
                                            const uint32_t *inst_emit, const uint32_t *tile_ranges,
                                            const uint32_t *tile_order, const gsr_camera *cams, int32_t n_views,
                                            const gsr_raster *r, const float *T_final, const uint32_t *n_contrib,
                                            const uint32_t *contrib_offsets, const uint32_t *contrib_ids,
                                            int64_t contrib_capacity, const float *dL_drgb, const float *dL_ddepth,
                                            float *dinst, gsr_stream stream) {
    if (!raster_ok(r) || n_views < 1 || !cams || !tile_ranges || !T_final || !n_contrib || !contrib_offsets ||
        !contrib_ids || !dL_drgb || !dinst || !inst_emit || !inst_gid || !splats)
        return GSR_E_INVALID;
    if (contrib_capacity < 1 || contrib_capacity >= (int64_t)UINT32_MAX) return GSR_E_INVALID;
    return gsr_render_bwd_stored_launch(splats, inst_gid, inst_emit, tile_ranges, tile_order, cams, n_views, r,
                                        T_final, n_contrib, contrib_offsets, contrib_ids, (uint32_t)contrib_capacity,
                                        dL_drgb, dL_ddepth, dinst, S(stream));
}

extern "C" gsr_status gsr_pair_grads(const float *dinst, const gsr_emission *em, const uint32_t *tile_info, int64_t n,
                                     int32_t n_views, float *dsplat, gsr_stream stream) {
    if (n < 0 || n_views < 1) return GSR_E_INVALID;
    if ((int64_t)n_views * n >= (int64_t)UINT32_MAX) return GSR_E_INVALID;
    if (n > 0 && (!dinst || !emission_ok(em) || !tile_info || !dsplat)) return GSR_E_INVALID;
    return gsr_pair_grads_launch(dinst, em, tile_info, (int64_t)n_views * n, dsplat, true, S(stream));
}

extern "C" gsr_status gsr_project_bwd(const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                      const gsr_raster *r, const gsr_splat *splats, const float *dinst,
                                      const gsr_emission *em, const uint32_t *tile_info, const gsr_param_grads *out, double *dpose, const int32_t *segment_id,
                                      int32_t min_segment, uint8_t *row_mask, void *ws, size_t ws_bytes,
                                      gsr_stream stream) {
    if (!gauss_ok(g) || !raster_ok(r) || n_views < 1 || !cams || !out) return GSR_E_INVALID;
    if ((int64_t)n_views * g->n >= (int64_t)UINT32_MAX) return GSR_E_INVALID;
    if (g->n > 0 && (!splats || !dinst || !emission_ok(em) || !tile_info || !out->means || !out->log_scales ||
                     !out->quats || !out->opacity_logits || !out->sh))
        return GSR_E_INVALID;
    if (g->n > 0 && (!ws || ws_bytes < gsr_project_bwd_workspace(g->n, n_views))) return GSR_E_CAPACITY;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return GSR_E_INVALID;
    return gsr_project_bwd_launch(g, cams, n_views, r, splats, dinst, em, out, dpose, tile_info, segment_id,
                                  min_segment, row_mask, nullptr, nullptr, nullptr, ws, S(stream));
}

extern "C" gsr_status gsr_project_bwd_adam(const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                           const gsr_raster *r, const gsr_splat *splats, const float *dinst,
                                           const gsr_emission *em, const uint32_t *tile_info,
                                           const uint32_t *visible_list, const uint32_t *visible_count,
                                           const int32_t *segment_id, int32_t min_segment,
                                           const gsr_adam_fused *adam, double *dpose, uint8_t *row_mask, void *ws,
                                           size_t ws_bytes, gsr_stream stream) {
    if ((visible_list == nullptr) != (visible_count == nullptr)) return GSR_E_INVALID;
    if (!gauss_ok(g) || !raster_ok(r) || n_views < 1 || !cams || !adam) return GSR_E_INVALID;
    if ((int64_t)n_views * g->n >= (int64_t)UINT32_MAX) return GSR_E_INVALID;
    if (g->n > 0 && (!splats || !dinst || !emission_ok(em) || !tile_info || !adam->step || !adam->m.means ||
                     !adam->m.log_scales || !adam->m.quats || !adam->m.opacity_logits || !adam->m.sh ||
                     !adam->v.means || !adam->v.log_scales || !adam->v.quats || !adam->v.opacity_logits ||
                     !adam->v.sh))
        return GSR_E_INVALID;
    if (!(adam->beta1 >= 0.f && adam->beta1 < 1.f && adam->beta2 >= 0.f && adam->beta2 < 1.f && adam->eps >= 0.f))
        return GSR_E_INVALID;
    if (g->n > 0 && (!ws || ws_bytes < gsr_project_bwd_workspace(g->n, n_views))) return GSR_E_CAPACITY;
    if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return GSR_E_INVALID;
    return gsr_project_bwd_launch(g, cams, n_views, r, splats, dinst, em, nullptr, dpose, tile_info,
                                  segment_id, min_segment, row_mask, adam, visible_list, visible_count, ws, S(stream));
}

extern "C" size_t gsr_visible_list_workspace(int64_t n) { return n < 0 ? 0 : gsr_visible_list_ws_bytes(n); }

extern "C" gsr_status gsr_visible_list(const uint32_t *tile_info, int64_t n, int32_t n_views, uint32_t *list,
                                       uint32_t *count, void *ws, size_t ws_bytes, gsr_stream stream) {
    if (n < 0 || n_views < 1 || !count || (n > 0 && (!tile_info || !list)) || !ws) return GSR_E_INVALID;
    if (ws_bytes < gsr_visible_list_ws_bytes(n)) return GSR_E_CAPACITY;
    return gsr_visible_list_launch(tile_info, n, n_views, list, count, ws, S(stream));
}

extern "C" gsr_status gsr_step_prep_launch(const gsr_camera *, int32_t, const int64_t *, int32_t, gsr_camera *,
                                           int32_t *, double *, int32_t *, uint8_t *, int64_t, hipStream_t);

extern "C" gsr_status gsr_step_prep(const gsr_camera *pool, int32_t n_pool, const int64_t *view_idx, int32_t n_views,
                                    gsr_camera *cams, int32_t *view_idx32, double *loss, int32_t *step,
                                    uint8_t *row_mask, int64_t n, gsr_stream stream) {
    if (!pool || n_pool < 1 || !view_idx || n_views < 1 || !cams || n < 0) return GSR_E_INVALID;
    if (reinterpret_cast<uintptr_t>(row_mask) & 15u) return GSR_E_INVALID;  // cleared 16 bytes per store
    return gsr_step_prep_launch(pool, n_pool, view_idx, n_views, cams, view_idx32, loss, step, row_mask, n,
                                S(stream));
}

extern "C" gsr_status gsr_adam_step(const gsr_adam_groups *groups, int64_t rows, const uint8_t *row_mask, float beta1,
                                    float beta2, float eps, int32_t step, gsr_stream stream) {
    if (!groups || groups->n_groups < 1 || groups->n_groups > GSR_MAX_GROUPS || rows < 0 || step < 1)
        return GSR_E_INVALID;
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f)) return GSR_E_INVALID;
    for (int k = 0; k < groups->n_groups; k++) {
        if (groups->cols[k] < 0) return GSR_E_INVALID;
        if (rows > 0 && groups->cols[k] > 0 &&
            (!groups->param[k] || !groups->grad[k] || !groups->m[k] || !groups->v[k]))
            return GSR_E_INVALID;
    }
    return gsr_adam_launch(groups, rows, row_mask, beta1, beta2, eps, step, S(stream));
}

extern "C" gsr_status gsr_loss_l1(const float *rgb, const float *depth, const float *target_rgb,
                                  const float *target_depth, const int32_t *target_index, int32_t n_views,
                                  const gsr_raster *r, float lambda_depth, double *loss, float *dL_drgb,
                                  float *dL_ddepth, gsr_stream stream) {
    if (!raster_ok(r) || n_views < 1 || !rgb || !target_rgb || !loss || !dL_drgb) return GSR_E_INVALID;
    if (target_depth && !depth) return GSR_E_INVALID;
    return gsr_loss_l1_launch(rgb, depth, target_rgb, target_depth, target_index, n_views, r, lambda_depth, loss,
                              dL_drgb, dL_ddepth, S(stream));
}

extern "C" gsr_status gsr_support_mask(const float *T_final, int32_t n_views, const gsr_raster *r, float tau_geo,
                                       int32_t r_erode, uint8_t *mask, uint32_t *count, gsr_stream stream) {
    if (!raster_ok(r) || n_views < 1 || !T_final || !mask || !count) return GSR_E_INVALID;
    if (!(tau_geo >= 0.0f && tau_geo <= 1.0f) || r_erode < 0 || r_erode > 8) return GSR_E_INVALID;
    return gsr_support_mask_launch(T_final, n_views, r, tau_geo, r_erode, mask, count, S(stream));
}

extern "C" size_t gsr_loss_workspace(int32_t n_views, const gsr_raster *r) {
    if (!raster_ok(r) || n_views < 1) return 0;
    return gsr_loss_ws_bytes(n_views, r);
}

extern "C" gsr_status gsr_loss(const float *rgb, const float *depth, const float *target_rgb, const float *target_depth,
                               const int32_t *target_index, int32_t n_views, const gsr_raster *r, const uint8_t *mask,
                               const uint32_t *count, float lambda_rgb, float lambda_ssim, float lambda_depth,
                               double *loss, float *dL_drgb, float *dL_ddepth, void *ws, size_t ws_bytes,
                               gsr_stream stream) {
    if (!raster_ok(r) || n_views < 1 || !rgb || !target_rgb || !loss || !dL_drgb) return GSR_E_INVALID;
    if (target_depth && !depth) return GSR_E_INVALID;
    if (mask && !count) return GSR_E_INVALID;
    if (!std::isfinite(lambda_rgb) || !std::isfinite(lambda_ssim) || !std::isfinite(lambda_depth)) return GSR_E_INVALID;
    if (!ws || ws_bytes < gsr_loss_ws_bytes(n_views, r)) return GSR_E_INVALID;
    return gsr_loss_launch(rgb, depth, target_rgb, target_depth, target_index, n_views, r, mask, count, lambda_rgb,
                           lambda_ssim, lambda_depth, loss, dL_drgb, dL_ddepth, ws, S(stream));
}

extern "C" size_t gsr_row_order_workspace(int64_t n) { return n < 0 ? 0 : gsr_row_order_ws_bytes(n); }

extern "C" gsr_status gsr_row_order(const float *means, const int32_t *segment_id, int64_t n, uint32_t *order,
                                    void *ws, size_t ws_bytes, gsr_stream stream) {
    if (n < 0 || n >= (int64_t)UINT32_MAX) return GSR_E_INVALID;
    if (n > 0 && (!means || !order || !ws)) return GSR_E_INVALID;
    if (ws_bytes < gsr_row_order_ws_bytes(n)) return GSR_E_CAPACITY;
    return gsr_row_order_launch(means, segment_id, n, order, ws, S(stream));
}

extern "C" size_t gsr_prune_workspace(int64_t n) { return n < 0 ? 0 : gsr_prune_ws_bytes(n); }

extern "C" gsr_status gsr_prune_select(const float *opacity_logits, const int32_t *segment_id, int32_t min_segment,
                                       int64_t n, float max_logit, float max_ratio, uint32_t *keep_index,
                                       uint32_t *n_keep, void *ws, size_t ws_bytes, gsr_stream stream) {
    if (n < 0 || n >= (int64_t)UINT32_MAX || !n_keep) return GSR_E_INVALID;
    if (!(max_ratio >= 0.0f && max_ratio <= 1.0f) || std::isnan(max_logit)) return GSR_E_INVALID;
    if (n > 0 && (!opacity_logits || !keep_index || !ws || ws_bytes < gsr_prune_ws_bytes(n))) return GSR_E_INVALID;
    const uint64_t budget = (uint64_t)floor((double)max_ratio * (double)n);
    return gsr_prune_launch(opacity_logits, segment_id, min_segment, n, max_logit, budget, keep_index, n_keep, ws,
                            S(stream));
}

extern "C" gsr_status gsr_gather_rows(const gsr_row_groups *groups, int64_t src_rows, const uint32_t *index,
                                      int64_t n_rows, int64_t dst_rows, int64_t dst_offset, gsr_stream stream) {
    if (!groups || groups->n_groups < 0 || groups->n_groups > GSR_MAX_ROW_GROUPS) return GSR_E_INVALID;
    if (src_rows < 0 || n_rows < 0 || dst_offset < 0 || dst_offset + n_rows > dst_rows) return GSR_E_INVALID;
    if (!index && n_rows > src_rows) return GSR_E_INVALID;
    for (int k = 0; k < groups->n_groups; k++)
        if (groups->cols[k] < 0 || (groups->cols[k] > 0 && n_rows > 0 && (!groups->src[k] || !groups->dst[k])))
            return GSR_E_INVALID;
    if (n_rows > 0 && index == nullptr && src_rows == 0) return GSR_E_INVALID;
    return gsr_gather_launch(groups, src_rows, index, n_rows, dst_rows, dst_offset, S(stream));
}

extern "C" size_t gsr_proximity_workspace(int64_t n_map, int64_t n_new) {
    return (n_map < 0 || n_new < 0) ? 0 : gsr_proximity_ws_bytes(n_map, n_new);
}

extern "C" gsr_status gsr_proximity_filter(const float *map_means, int64_t n_map, const float *new_means,
                                           int64_t n_new, float d_min, uint8_t *keep, uint32_t *keep_index,
                                           uint32_t *n_keep, void *ws, size_t ws_bytes, gsr_stream stream) {
    if (n_map < 0 || n_new < 0 || n_map >= (int64_t)UINT32_MAX || n_new >= (int64_t)UINT32_MAX || !n_keep)
        return GSR_E_INVALID;
    if (!(d_min > 0.0f) || !std::isfinite(d_min)) return GSR_E_INVALID;
    if (n_map > 0 && !map_means) return GSR_E_INVALID;
    if (n_new > 0 && (!new_means || !keep || !keep_index || !ws || ws_bytes < gsr_proximity_ws_bytes(n_map, n_new)))
        return GSR_E_INVALID;
    return gsr_proximity_launch(map_means, n_map, new_means, n_new, d_min, keep, keep_index, n_keep, ws, S(stream));
}

extern "C" size_t gsr_gicp_workspace(int64_t n) { return n < 0 ? 0 : gsr_gicp_ws_bytes(n); }

namespace {
bool gicp_gauss_ok(const gsr_gaussians *g) {
    return g && g->n >= 0 && g->n < (int64_t)UINT32_MAX && (g->n == 0 || (g->means && g->quats && g->log_scales));
}
}  // namespace

extern "C" gsr_status gsr_gicp_prepare(const gsr_gaussians *g, const int32_t *segment_id, int32_t src_segment,
                                       const gsr_camera *cams, int32_t n_cams, float d_max, float d_corr,
                                       uint32_t *src_index, uint32_t *tgt_index, uint32_t *counts, double *stats,
                                       void *ws, size_t ws_bytes, gsr_stream stream) {
    if (!gicp_gauss_ok(g) || !counts || !stats || n_cams < 0 || (n_cams > 0 && !cams)) return GSR_E_INVALID;
    if (!(d_max > 0.0f) || !(d_corr > 0.0f) || !std::isfinite(d_max) || !std::isfinite(d_corr)) return GSR_E_INVALID;
    if (g->n > 0 && (!segment_id || !src_index || !tgt_index || !ws || ws_bytes < gsr_gicp_ws_bytes(g->n)))
        return GSR_E_INVALID;
    return gsr_gicp_prepare_launch(g, segment_id, src_segment, cams, n_cams, d_max, d_corr, src_index, tgt_index,
                                   counts, stats, ws, S(stream));
}

extern "C" gsr_status gsr_gicp_iterate(const gsr_gaussians *g, const uint32_t *src_index, const uint32_t *tgt_index,
                                       const uint32_t *counts, float d_corr, double *pose, double *stats,
                                       int32_t *corr, int32_t n_iter, void *ws, size_t ws_bytes, gsr_stream stream) {
    if (!gicp_gauss_ok(g) || !counts || !pose || !stats || n_iter < 0) return GSR_E_INVALID;
    if (!(d_corr > 0.0f) || !std::isfinite(d_corr)) return GSR_E_INVALID;
    if (g->n > 0 && (!src_index || !tgt_index || !ws || ws_bytes < gsr_gicp_ws_bytes(g->n))) return GSR_E_INVALID;
    return gsr_gicp_iterate_launch(g, src_index, tgt_index, counts, d_corr, pose, stats, corr, n_iter, ws, S(stream));
}

extern "C" gsr_status gsr_transform_segment(const gsr_params *p, int64_t n, int32_t sh_degree,
                                            const int32_t *segment_id, int32_t segment, const double *pose, double *ws,
                                            gsr_stream stream) {
    if (!p || n < 0 || sh_degree < 0 || sh_degree > 3 || !pose || !ws) return GSR_E_INVALID;
    if (n > 0 && (!p->means || !p->quats || !segment_id || (sh_degree > 0 && !p->sh))) return GSR_E_INVALID;
    return gsr_transform_segment_launch(p, n, sh_degree, segment_id, segment, pose, ws, S(stream));
}

extern "C" gsr_status gsr_transform_cameras(gsr_camera *cams, int32_t n_cams, const uint8_t *mask, const double *pose,
                                           gsr_stream stream) {
    if (n_cams < 0 || (n_cams > 0 && !cams) || !pose) return GSR_E_INVALID;
    return gsr_transform_cameras_launch(cams, n_cams, mask, pose, S(stream));
}

extern "C" gsr_status gsr_fill_u32(void *dst, uint32_t value, int64_t n_words, gsr_stream stream) {
    if (n_words < 0 || (n_words > 0 && !dst)) return GSR_E_INVALID;
    return gsr_fill_u32_launch(dst, value, n_words, S(stream));
}

extern "C" size_t gsr_voxel_pca_workspace(int64_t n) { return n < 0 ? 0 : gsr_voxel_pca_ws_bytes(n); }

extern "C" gsr_status gsr_voxel_pca(const float *points, int64_t n, uint64_t seed, const gsr_voxels *out, void *ws,
                                    size_t ws_bytes, gsr_stream stream) {
    if (n < 0 || n >= (int64_t)UINT32_MAX || !out || !out->n_voxels || !out->n_outside) return GSR_E_INVALID;
    if (n > 0 && (!points || !out->key || !out->start || !out->count || !out->point_order || !out->point_voxel ||
                  !out->mu || !out->evals || !out->R || !out->s_pca || !out->trace || !out->cls || !out->reliable ||
                  !ws))
        return GSR_E_INVALID;
    if (n > 0 && (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return GSR_E_INVALID;
    if (n > 0 && ws_bytes < gsr_voxel_pca_ws_bytes(n)) return GSR_E_CAPACITY;
    return gsr_voxel_pca_launch(points, n, seed, out, ws, S(stream));
}

extern "C" gsr_status gsr_voxel_pca_cov(const float *points, const float *point_cov, int64_t n, uint64_t seed,
                                        const gsr_voxels *out, float *sigma_g, void *ws, size_t ws_bytes,
                                        gsr_stream stream) {
    if (n > 0 && !point_cov) return GSR_E_INVALID;
    if (n < 0 || n >= (int64_t)UINT32_MAX || !out || !out->n_voxels || !out->n_outside) return GSR_E_INVALID;
    if (n > 0 && (!points || !out->key || !out->start || !out->count || !out->point_order || !out->point_voxel ||
                  !out->mu || !out->evals || !out->R || !out->s_pca || !out->trace || !out->cls || !out->reliable ||
                  !ws))
        return GSR_E_INVALID;
    if (n > 0 && (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return GSR_E_INVALID;
    if (n > 0 && ws_bytes < gsr_voxel_pca_ws_bytes(n)) return GSR_E_CAPACITY;
    return gsr_voxel_pca_cov_launch(points, point_cov, n, seed, out, sigma_g, ws, S(stream));
}

extern "C" size_t gsr_cascade_workspace(int32_t n_segments) { return gsr_cascade_ws_bytes(n_segments); }

extern "C" gsr_status gsr_cascade(const float *points, const float *colors, const float *depth, const int32_t *segment,
                                  int32_t n_segments, int64_t n, const gsr_voxels *vox, const float *pred, float focal,
                                  float beta, int32_t sh_degree, const gsr_params *out, uint8_t *branch, void *ws,
                                  size_t ws_bytes, gsr_stream stream) {
    if (n < 0 || n >= (int64_t)UINT32_MAX || sh_degree < 0 || sh_degree > 3 || !vox || !out) return GSR_E_INVALID;
    if (segment && n_segments < 1) return GSR_E_INVALID;
    if (n > 0 && (!points || !colors || !depth || !vox->point_voxel || !vox->reliable || !vox->s_pca || !vox->R ||
                  !out->means || !out->log_scales || !out->quats || !out->opacity_logits || !out->sh || !branch || !ws))
        return GSR_E_INVALID;
    if (!(focal > 0.f)) return GSR_E_INVALID;
    if (ws_bytes < gsr_cascade_ws_bytes(segment ? n_segments : 1)) return GSR_E_CAPACITY;
    return gsr_cascade_launch(points, colors, depth, segment, segment ? n_segments : 1, n, vox, pred, focal, beta,
                              sh_degree, out, branch, ws, S(stream), 0);
}

extern "C" gsr_status gsr_cascade_anchored(const float *points, const float *colors, const float *depth,
                                           const int32_t *segment, int32_t n_segments, int64_t n,
                                           const gsr_voxels *vox, const float *pred, float focal, float beta,
                                           int32_t sh_degree, const gsr_params *out, uint8_t *branch, void *ws,
                                           size_t ws_bytes, gsr_stream stream) {
    if (n < 0 || n >= (int64_t)UINT32_MAX || sh_degree < 0 || sh_degree > 3 || !vox || !out) return GSR_E_INVALID;
    if (segment && n_segments < 1) return GSR_E_INVALID;
    if (n > 0 && (!points || !colors || !depth || !vox->point_voxel || !vox->reliable || !vox->s_pca || !vox->R ||
                  !out->means || !out->log_scales || !out->quats || !out->opacity_logits || !out->sh || !branch || !ws))
        return GSR_E_INVALID;
    if (!(focal > 0.f)) return GSR_E_INVALID;
    if (ws_bytes < gsr_cascade_ws_bytes(segment ? n_segments : 1)) return GSR_E_CAPACITY;
    return gsr_cascade_launch(points, colors, depth, segment, segment ? n_segments : 1, n, vox, pred, focal, beta,
                              sh_degree, out, branch, ws, S(stream), 1);
}

namespace {
bool voxels_ok(const gsr_voxels *v) {
    return v && v->n_voxels && v->count && v->start && v->point_order && v->mu && v->evals && v->R;
}
}  // namespace

extern "C" gsr_status gsr_pointnet_fwd(const float *points, int64_t n, const gsr_voxels *vox, const float *weights,
                                       float *y, gsr_stream stream) {
    if (n < 0 || n >= (int64_t)UINT32_MAX || !voxels_ok(vox)) return GSR_E_INVALID;
    if (n > 0 && (!points || !weights || !y)) return GSR_E_INVALID;
    return gsr_pointnet_fwd_launch(points, n, vox, weights, y, S(stream));
}

extern "C" size_t gsr_pointnet_bwd_workspace(int32_t blocks) { return blocks < 1 ? 0 : gsr_pointnet_bwd_ws_bytes(blocks); }

extern "C" gsr_status gsr_pointnet_bwd(const float *points, int64_t n, const gsr_voxels *vox, const float *weights,
                                       const float *cov_t, const float *o_t, const uint8_t *tmask, float inv_count,
                                       int32_t blocks, float *grad, double *loss, void *ws, size_t ws_bytes,
                                       gsr_stream stream) {
    if (n < 0 || n >= (int64_t)UINT32_MAX || !voxels_ok(vox) || blocks < 1 || blocks > 65536) return GSR_E_INVALID;
    if (!points || !weights || !cov_t || !o_t || !grad || !loss || !ws) return GSR_E_INVALID;
    if (ws_bytes < gsr_pointnet_bwd_ws_bytes(blocks)) return GSR_E_CAPACITY;
    return gsr_pointnet_bwd_launch(points, n, vox, weights, cov_t, o_t, tmask, inv_count, blocks, grad, loss, ws,
                                   S(stream));
}


extern "C" gsr_status gsr_voxel_targets(const gsr_params *gauss, int64_t n, const gsr_voxels *vox, float *cov_t,
                                       float *o_t, uint8_t *has, gsr_stream stream) {
    if (n < 0 || n >= (int64_t)UINT32_MAX || !gauss || !vox) return GSR_E_INVALID;
    if (n > 0 && (!gauss->log_scales || !gauss->quats || !gauss->opacity_logits || !vox->n_voxels || !vox->start ||
                  !vox->count || !vox->point_order || !cov_t || !o_t || !has))
        return GSR_E_INVALID;
    return gsr_voxel_targets_launch(gauss, n, vox, cov_t, o_t, has, S(stream));
}
