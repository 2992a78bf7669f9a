/*
 * gsr.h -- C ABI of the MI355X (gfx950) differentiable Gaussian-splatting rasterizer that
 * drives the global Gaussian-map optimisation of RMGS-SLAM (arXiv 2604.12942, Sec. III-C
 * "Optimization").  The paper renders colour by standard differentiable splatting with
 * front-to-back alpha compositing, renders depth with the same compositing weights
 * (Eq. 8), supervises with masked L1 colour / depth terms (Eq. 9, 10, 12) and refines the
 * visible, unfrozen Gaussians with a sparse gradient optimiser.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller.  The library never
 *    allocates, frees or synchronises; all work is enqueued on the caller's stream.  Struct
 *    arguments passed by pointer (gsr_gaussians, gsr_raster, ...) are HOST structs that hold
 *    device pointers; they are read before the call returns.
 *  - Gaussian parameters are structure-of-arrays, component-major [c][n] float32:
 *      means [3][n], log_scales [3][n], quats [4][n] as raw (w, x, y, z), opacity_logits [n],
 *      sh [3K][n] with row k*3+ch (K = (sh_degree+1)^2, real SH without Condon-Shortley
 *      phase, ordered (l, m = -l..l), colour = max(0, sum_k Y_k(d) sh_k + 1/2)).
 *  - Cameras: a device array of gsr_camera, world->camera p = R mu + t, camera looking along
 *    +z, image x right and y down; every view of a call shares gsr_raster's width / height.
 *    Pixel (i, j) is sampled at its centre (i + 1/2, j + 1/2).
 *  - "Projected splat" records are 48-byte gsr_splat structs, one per (view, Gaussian), at
 *    index v*n + i.
 *  - Errors: invalid arguments return GSR_E_INVALID before any launch; a failed launch returns
 *    GSR_E_HIP.  No C++ exception crosses this interface.  Capacity overflow of the instance
 *    buffer is detected on the device (see gsr_bin_sort).
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSR_ABI_VERSION 4
#define GSR_API __attribute__((visibility("default")))

typedef enum {
    GSR_OK = 0,
    GSR_E_INVALID = 1,     /* bad argument, nothing launched */
    GSR_E_CAPACITY = 2,    /* a caller-provided workspace is too small */
    GSR_E_HIP = 3,         /* a HIP launch or runtime call failed */
    GSR_E_UNSUPPORTED = 4  /* configuration the library does not handle */
} gsr_status;

typedef void *gsr_stream; /* a hipStream_t (NULL = the null stream) */

/* One camera, 96 bytes.  R row-major world->camera rotation, t translation, pinhole
   intrinsics, near plane (Gaussians with camera z <= z_near are culled) and background. */
typedef struct {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float z_near;
    float bg[3];
    int32_t width, height; /* must equal the gsr_raster of the call */
    int32_t _pad[2];
} gsr_camera;

typedef struct {
    const float *means, *log_scales, *quats, *opacity_logits, *sh;
    int64_t n;
    int32_t sh_degree; /* 0..3 */
    int32_t _pad;
} gsr_gaussians;

typedef struct {
    float *means, *log_scales, *quats, *opacity_logits, *sh;
} gsr_param_grads; /* same layouts as gsr_gaussians; ACCUMULATED into */

/* Image size shared by the views of a call and the screen tile shape.  Supported tile
   shapes (tile_w x tile_h): 16x16, 8x32, 32x8.  Images are identical for every shape. */
typedef struct {
    int32_t width, height;
    int32_t tile_w, tile_h;
} gsr_raster;

/* Projected splat of one (view, Gaussian): 48 bytes.
     u, v      pixel-space mean (double so a tile can re-centre it without rounding loss)
     l11,l21,l22  lower Cholesky factor L of (log2(e)/2) * Q, Q = inverse screen covariance:
               the blend weight exponent at offset D is |L^T D|^2, alpha = o * 2^-(|L^T D|^2)
     opacity   o = sigmoid(logit)
     depth     camera-frame z (ordering key and Eq. 8 depth)
     r, g, b   view-dependent colour after the clamp at 0                                  */
typedef struct {
    double u, v;
    float l11, l21, l22;
    float opacity;
    float depth;
    float r, g, b;
} gsr_splat;

/* Screen-space gradient of one (view, Gaussian), 10 floats in this order:
   dL/du, dL/dv, dL/dQa, dL/dQb, dL/dQc (Q = [[Qa, Qb], [Qb, Qc]], Qb counted once),
   dL/do, dL/dr, dL/dg, dL/db, dL/dz. */
#define GSR_SPLAT_GRAD_FLOATS 10

GSR_API int gsr_abi_version(void);
GSR_API const char *gsr_status_str(int status);

/* Number of screen tiles per view for a raster. */
GSR_API int64_t gsr_tiles_per_view(const gsr_raster *r);

/* ---- project ---------------------------------------------------------------------------------
 * EWA projection of every Gaussian into every view (Sec. III-C: standard splatting; Eq. 8's
 * camera-frame depth).  Per (view v, Gaussian i): p = R mu + t; culled if z <= z_near;
 * Sigma = Rq S S^T Rq^T, Sigma' = J R Sigma R^T J^T + 0.3 I with the perspective Jacobian J
 * (x/z, y/z clamped to 1.3x the half field of view), Q = Sigma'^-1, opacity sigmoid, SH colour
 * in the viewing direction from the camera centre -R^T t.  A pair contributes to a pixel iff
 * o exp(-D^T Q D / 2) >= 1/255, so the footprint is the ellipse D^T Q D <= 2 ln(255 o).
 * Outputs:  splats [V*n] gsr_splat;  tile_info uint32 [4][V*n] (component-major):
 *   row 0  n_tiles: number of tiles the pair is emitted to (0 = not visible in that view)
 *   row 1  depth key: the float32 bit pattern of the camera-frame depth (monotone for z > 0)
 *   row 2  tx0 | ty0 << 16, row 3  tx1 | ty1 << 16: inclusive tile rectangle that
 *          conservatively covers every pixel centre of the footprint.
 * cams: device [n_views].  Errors: GSR_E_INVALID for NULL pointers, n < 0, sh_degree outside
 * 0..3, n_views < 1, width/height <= 0, an unsupported tile shape, or V*n >= 2^32. */
GSR_API gsr_status gsr_project(const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views, const gsr_raster *r,
                       gsr_splat *splats, uint32_t *tile_info, gsr_stream stream);

/* ---- bin / sort ------------------------------------------------------------------------------
 * Tile binning with a radix sort on (tile, depth) keys.  Emits one instance per (view, tile,
 * Gaussian) that project's rectangle covers and orders them lexicographically by
 * (view, tile index ty*ntx+tx, float32 depth bits, Gaussian index): visible pairs are first
 * radix-sorted stably by depth bits (index order breaks ties), then instances are emitted in
 * that order ("emission order": a pair's tiles row-major and consecutive) and radix-sorted
 * stably by (view, tile).  Outputs, all device memory:
 *   inst_gid    [capacity]  v*n + i of each instance, in sorted order
 *   tile_ranges [V*T][2]    [start, end) of each view-tile's instances
 *   *n_instances            (uint32) the REQUIRED instance count M.
 * If M > capacity the lists would be incomplete, so the call leaves a frame in which nothing is
 * visible instead: row 0 of tile_info is cleared (which is why tile_info is not const), every
 * tile range is empty and em->n_pairs is 0.  Everything later in the step then does nothing:
 * the renders write background images, the backward zero gradients and no pose gradient, and the
 * fused Adam and the visible list find no row; no kernel reads past the capacity.  *n_instances
 * still receives M: the caller compares it with capacity after synchronising, grows the buffers
 * and runs gsr_project and gsr_bin_sort again (a captured step is captured again).
 * tile_order (device uint32 [V*T], may be NULL) receives the view-tiles sorted by descending
 * instance count resolved to 1/16 of an octave (counts c with the same floor(log2 c) and the same
 * four bits below the leading one tie; empty tiles tie with single-instance ones, and counts of
 * 2^16 and more with the top step below 2^16; ties by index): the
 * longest-processing-time-first launch order the render kernels use to keep heavy tiles off the
 * tail of the grid.
 * em (may be NULL; needed by the backward) receives the emission bookkeeping, see gsr_emission.
 * ws: device workspace of at least gsr_bin_sort_workspace(n, n_views, capacity, r) bytes,
 * 256-byte aligned.  Errors: GSR_E_INVALID (bad pointers or sizes, capacity >= 2^32),
 * GSR_E_CAPACITY (ws_bytes too small). */
typedef struct {
    uint32_t *inst_emit;  /* [capacity]: emission index of each sorted instance (where
                             gsr_render_bwd stores its gradient record)                      */
    uint32_t *pair_gid;   /* [V*n]: the visible pairs (v*n + i) in emission order             */
    uint32_t *pair_first; /* [V*n]: emission index of each listed pair's first instance; the
                             pair has tile_info row 0 many instances                          */
    uint32_t *n_pairs;    /* [1]: number of listed pairs                                      */
} gsr_emission;
GSR_API size_t gsr_bin_sort_workspace(int64_t n, int32_t n_views, int64_t capacity, const gsr_raster *r);
GSR_API gsr_status gsr_bin_sort(uint32_t *tile_info, int64_t n, int32_t n_views, const gsr_raster *r,
                                uint32_t *inst_gid, const gsr_emission *em, int64_t capacity,
                                uint32_t *tile_ranges, uint32_t *n_instances, uint32_t *tile_order, void *ws,
                                size_t ws_bytes, gsr_stream stream);

/* ---- render forward --------------------------------------------------------------------------
 * Front-to-back alpha compositing per pixel (Sec. III-C; Eq. 8).  For each view-tile's
 * instances in order: a = min(0.99, alpha), skipped if alpha < 1/255; T' = T (1 - a); the
 * pixel stops when T' < 1e-4 (that Gaussian is not composited); C += a T rgb, D += a T z.
 * Outputs (images [V][...][H][W]): rgb [V][3][H][W] = C + T bg, depth [V][H][W] = D (no
 * background term), T_final [V][H][W], last [V][H][W] = number of the tile's instances up to
 * and including the pixel's last composited one (the backward re-walks exactly these), and,
 * if n_contrib is not NULL, n_contrib [V][H][W] = the number of composited Gaussians.
 * tile_order (from gsr_bin_sort, may be NULL = natural order) only sets the launch order. */
GSR_API gsr_status gsr_render_fwd(const gsr_splat *splats, const uint32_t *inst_gid, const uint32_t *tile_ranges,
                          const uint32_t *tile_order, const gsr_camera *cams, int32_t n_views, const gsr_raster *r, float *rgb, float *depth,
                          float *T_final, uint32_t *last, uint32_t *n_contrib, gsr_stream stream);

/* ---- render forward with depth slices ------------------------------------------------------------
 * The same outputs as gsr_render_fwd (n_contrib excepted) with the long tiles split.  A view-tile
 * whose list holds more than 8192 instances is cut into slices of 1024 consecutive instances,
 * composited by separate workgroups: a first pass forms each slice's per-pixel product of
 * (1 - a); every slice k then starts from T_in(k), the product over the slices in front of it,
 * and does nothing for a pixel with T_in(k) < 1e-4 (already terminated); a last pass adds the
 * pixel's slice results in order up to the slice where it terminated.  This is the front-to-back
 * recurrence of Eq. 8 regrouped by the associativity of the transmittance product: results equal
 * gsr_render_fwd's up to the float rounding of those products, so images are no longer
 * bit-identical across tile shapes for the split tiles.  Tiles of at most 8192 instances are
 * composited exactly as by gsr_render_fwd.
 * capacity: the instance capacity the lists were built with (gsr_bin_sort's), which bounds the
 * number of slices.  ws: device workspace of gsr_render_fwd_sliced_workspace(V, r, capacity)
 * bytes (about 7.7 KiB per 1,000 instances of capacity), 256-byte aligned.  After the call ws
 * holds, per slice and pixel, the transmittance behind the slice and the colour and depth
 * composited behind it: gsr_render_bwd and gsr_render_bwd_l1 given this ws run the backward of
 * the split tiles in the same slices.  Errors: GSR_E_INVALID, GSR_E_CAPACITY (ws_bytes too
 * small). */
GSR_API size_t gsr_render_fwd_sliced_workspace(int32_t n_views, const gsr_raster *r, int64_t capacity);
GSR_API gsr_status gsr_render_fwd_sliced(const gsr_splat *splats, const uint32_t *inst_gid,
                                         const uint32_t *tile_ranges, const uint32_t *tile_order,
                                         const gsr_camera *cams, int32_t n_views, const gsr_raster *r, float *rgb,
                                         float *depth, float *T_final, uint32_t *last, int64_t capacity, void *ws,
                                         size_t ws_bytes, gsr_stream stream);

/* ---- stored contributor lists ------------------------------------------------------------------
 * The alternative to re-walking the tile lists in the backward: the forward keeps, per pixel, the
 * list of the Gaussians it composited (memory for compute).  gsr_render_fwd_stored writes every
 * output of gsr_render_fwd (images, last, n_contrib [V][H][W] required) and, by a second pass over
 * the tiles after an exclusive scan of n_contrib:
 *   contrib_offsets [V][H][W]  (uint32) exclusive prefix sums of n_contrib in (v, y, x) order
 *   contrib_ids [contrib_capacity] (uint32) each pixel's composited Gaussians, front to back, as
 *                              positions in its view-tile's instance list (instance =
 *                              tile_ranges start + position)
 *   *n_contrib_total           (device uint32) the REQUIRED list size (must stay below 2^32).
 * Entries beyond contrib_capacity are not written: the caller compares *n_contrib_total with the
 * capacity after synchronising and calls again with more room.  ws:
 * gsr_render_fwd_stored_workspace(V, r) bytes (the scan's block sums).
 * gsr_render_bwd_stored computes exactly what gsr_render_bwd does (same dinst records), walking
 * each pixel's own list instead of the tile list; pixels whose list did not fit the capacity get
 * no gradient, so it must only be called after a forward whose lists fit. */
GSR_API size_t gsr_render_fwd_stored_workspace(int32_t n_views, const gsr_raster *r);
GSR_API gsr_status gsr_render_fwd_stored(const gsr_splat *splats, const uint32_t *inst_gid, const uint32_t *tile_ranges,
                                         const uint32_t *tile_order, const gsr_camera *cams, int32_t n_views,
                                         const gsr_raster *r, float *rgb, float *depth, float *T_final,
                                         uint32_t *last, uint32_t *n_contrib, uint32_t *contrib_offsets,
                                         uint32_t *contrib_ids, int64_t contrib_capacity, uint32_t *n_contrib_total,
                                         void *ws, size_t ws_bytes, gsr_stream stream);
GSR_API gsr_status gsr_render_bwd_stored(const gsr_splat *splats, const uint32_t *inst_gid, const uint32_t *inst_emit,
                                         const uint32_t *tile_ranges, const uint32_t *tile_order,
                                         const gsr_camera *cams, int32_t n_views, const gsr_raster *r,
                                         const float *T_final, const uint32_t *n_contrib,
                                         const uint32_t *contrib_offsets, const uint32_t *contrib_ids,
                                         int64_t contrib_capacity, const float *dL_drgb, const float *dL_ddepth,
                                         float *dinst, gsr_stream stream);

/* ---- render backward -------------------------------------------------------------------------
 * Exact gradient of the forward's outputs (every discrete decision held) given dL/drgb
 * [V][3][H][W] and dL/ddepth [V][H][W] (may be NULL).  Walks each pixel's instances back to
 * front, recovering transmittance by division.  For EVERY instance k < M of gsr_bin_sort it
 * stores, at dinst[inst_emit[k]][0..9] (inst_emit = gsr_emission.inst_emit) (float32 [capacity][GSR_SPLAT_GRAD_FLOATS]), the
 * screen-space gradient that its tile's pixels give its (view, Gaussian) pair: plain stores, no
 * accumulation and no clearing needed.  A pair's gradient is the sum of its instances' records
 * (gsr_pair_grads, or inside gsr_project_bwd), taken in a fixed order.  Each record, though, is
 * the sum of its tile's pixel terms formed by the four waves of a workgroup, whose adds into
 * shared memory come in an order that varies from run to run: gradients repeat from run to run
 * only up to float32 rounding, not bit for bit.
 * fwd_ws: NULL, or the workspace (fwd_ws_bytes long, 256-byte aligned) of the gsr_render_fwd_sliced
 * call, with this capacity and these lists, that produced T_final and last.  Then each view-tile
 * that forward composited in depth slices also runs its backward in those slices, one workgroup per
 * slice, each starting from the transmittance behind its slice and the colour and depth composited
 * behind it, which that forward's slice merge leaves in fwd_ws (read, not changed): the records
 * equal those of the whole-tile walk up to float rounding, and a long tile no longer holds one
 * workgroup for the whole launch.  Errors: GSR_E_INVALID (NULL pointers, a misaligned fwd_ws, a bad
 * capacity), GSR_E_CAPACITY (fwd_ws_bytes too small). */
GSR_API gsr_status gsr_render_bwd(const gsr_splat *splats, const uint32_t *inst_gid, const uint32_t *inst_emit,
                                  const uint32_t *tile_ranges, const uint32_t *tile_order, const gsr_camera *cams,
                                  int32_t n_views, const gsr_raster *r, const float *T_final, const uint32_t *last,
                                  const float *dL_drgb, const float *dL_ddepth, float *dinst, void *fwd_ws,
                                  size_t fwd_ws_bytes, int64_t capacity, gsr_stream stream);

/* ---- render backward of the per-pixel L1 loss ---------------------------------------------------
 * gsr_loss_l1 followed by gsr_render_bwd in one launch: each workgroup forms its view-tile's pixel
 * terms L_v = (1/P) sum_ch |C - C~| + lambda_depth (1/P) |D - D~| and gradients sign(C - C~)/P,
 * lambda_depth sign(D - D~)/P (sign(0) = 0) from the forward's rgb and depth and the targets in
 * registers (no gradient image is written or read), then writes the tile's backward records
 * exactly as gsr_render_bwd does for that upstream gradient (Sec. III-C, Eq. 8-10).  Inputs as
 * gsr_render_bwd plus the forward's rgb [V][3][H][W] and depth [V][H][W]; targets as gsr_loss_l1.
 * *loss (device float64) is ACCUMULATED, summed over the view-tiles in a fixed order.  ws:
 * gsr_render_bwd_l1_workspace(V, r) bytes (one float64 per view-tile), 256-byte aligned.
 * fwd_ws, fwd_ws_bytes, capacity: as for gsr_render_bwd (the sliced forward that produced rgb,
 * depth, T_final and last; its depth slices then carry the long tiles' backward; NULL: whole
 * tiles).  Errors: GSR_E_INVALID (NULL pointers, lambda_depth < 0, a misaligned ws or fwd_ws, a
 * bad capacity), GSR_E_CAPACITY (ws_bytes or fwd_ws_bytes too small). */
GSR_API size_t gsr_render_bwd_l1_workspace(int32_t n_views, const gsr_raster *r);
GSR_API gsr_status gsr_render_bwd_l1(const gsr_splat *splats, const uint32_t *inst_gid, const uint32_t *inst_emit,
                                     const uint32_t *tile_ranges, const uint32_t *tile_order, const gsr_camera *cams,
                                     int32_t n_views, const gsr_raster *r, const float *rgb, const float *depth,
                                     const float *T_final, const uint32_t *last, const float *target_rgb,
                                     const float *target_depth, const int32_t *target_index, float lambda_depth,
                                     double *loss, float *dinst, void *ws, size_t ws_bytes, void *fwd_ws,
                                     size_t fwd_ws_bytes, int64_t capacity, gsr_stream stream);

/* ---- fused step: render forward, L1 loss and render backward in one persistent launch ----------
 * The batched optimisation step of Sec. III-C with the loss of Eq. 9-10 restricted to its
 * per-pixel terms (all-ones mask, lambda_ssim = 0): for every view-tile, the front-to-back
 * compositing of gsr_render_fwd_sliced, then L_v = (1/P) sum_x sum_ch |C - C~| + lambda_depth
 * (1/P) sum_x |D - D~| with dL/dC = sign(C - C~)/P, dL/dD = lambda_depth sign(D - D~)/P
 * (sign(0) = 0), then the records of gsr_render_bwd for that upstream gradient.  One workgroup
 * takes a view-tile through all three, so the images and the loss gradient stay on chip between
 * the forward and the backward.  Work items come from a device queue: the depth slices of the long
 * tiles first (as in gsr_render_fwd_sliced; the workgroup that completes a tile's last slice
 * merges them and runs that tile's loss and backward), then the view-tiles in tile_order
 * (longest first; NULL = natural order).  Results equal those of gsr_render_fwd_sliced,
 * gsr_loss_l1 and gsr_render_bwd called in turn (images and loss gradient bit for bit, records up
 * to the float rounding of their four-wave LDS sums).
 * Inputs as gsr_render_fwd_sliced and gsr_render_bwd; targets as gsr_loss_l1 (target_rgb
 * [S][3][H][W], target_depth [S][H][W] or NULL, target_index [V] or NULL = slot v).  Outputs:
 * rgb, depth, T_final, last as gsr_render_fwd; *loss (device float64) ACCUMULATED, summed over the
 * view-tiles in a fixed order; dinst as gsr_render_bwd.  capacity: the instance capacity of the
 * lists.  ws: gsr_render_step_workspace(V, r, capacity) bytes, 256-byte aligned (the slice
 * workspace plus per view-tile loss sums and the queue counters, cleared by the call itself).
 * Errors: GSR_E_INVALID (NULL pointers, bad sizes, lambda_depth < 0), GSR_E_CAPACITY (ws_bytes
 * too small), GSR_E_HIP. */
GSR_API size_t gsr_render_step_workspace(int32_t n_views, const gsr_raster *r, int64_t capacity);
GSR_API gsr_status gsr_render_step(const gsr_splat *splats, const uint32_t *inst_gid, const uint32_t *inst_emit,
                                   const uint32_t *tile_ranges, const uint32_t *tile_order, const gsr_camera *cams,
                                   int32_t n_views, const gsr_raster *r, const float *target_rgb,
                                   const float *target_depth, const int32_t *target_index, float lambda_depth,
                                   float *rgb, float *depth, float *T_final, uint32_t *last, double *loss,
                                   float *dinst, int64_t capacity, void *ws, size_t ws_bytes, gsr_stream stream);

/* Screen-space gradient per (view, Gaussian): dsplat [V*n][10] (OVERWRITTEN) = the sum, in
 * emission order, of the pair's instance records in dinst (from gsr_render_bwd); the pairs and
 * their first records come from em (gsr_bin_sort): a pair's records end where the next pair's
 * begin, and the last pair's count is its tile count in tile_info row 0 (gsr_project); zero for
 * pairs that were not rendered. */
GSR_API gsr_status gsr_pair_grads(const float *dinst, const gsr_emission *em, const uint32_t *tile_info, int64_t n,
                                  int32_t n_views, float *dsplat, gsr_stream stream);

/* ---- project backward ------------------------------------------------------------------------
 * Chain rule from the screen-space gradients to every parameter, summed over views, plus the
 * per-view camera-pose gradient for a left perturbation T <- Exp(xi) T, xi = (rho, phi)
 * (translation first): p -> p + rho + phi x p.  The screen-space gradient of each rendered pair
 * (tile_info row 0 > 0) is the sum of its instance records dinst (gsr_render_bwd), located by
 * em (gsr_bin_sort); tile_info is the one gsr_project wrote.  Gradients are
 * ACCUMULATED into out; dpose [V][6] (float64, may be NULL) is OVERWRITTEN.  splats: the records
 * gsr_project wrote for these parameters (their clamped colours fix the colour clamp
 * decisions).  ws: device workspace of gsr_project_bwd_workspace(n, V) bytes, 256-byte aligned,
 * required when n > 0 (it holds the per-pair sums of the instance records and the pose
 * partials; GSR_E_CAPACITY if smaller).
 * Optional sparse-update mask (Sec. III-C: only visible Gaussians of the latest segments are
 * updated): if row_mask [n] is not NULL it receives 1 for Gaussians that are visible in at
 * least one view and whose segment_id [n] is >= min_segment (segment_id NULL = no freezing),
 * else 0. */
GSR_API size_t gsr_project_bwd_workspace(int64_t n, int32_t n_views);
GSR_API gsr_status gsr_project_bwd(const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                   const gsr_raster *r, const gsr_splat *splats, const float *dinst,
                                   const gsr_emission *em, const uint32_t *tile_info, const gsr_param_grads *out,
                                   double *dpose, const int32_t *segment_id, int32_t min_segment, uint8_t *row_mask,
                                   void *ws, size_t ws_bytes, gsr_stream stream);

/* ---- project backward fused with sparse Adam ---------------------------------------------------
 * The optimisation step's form of gsr_project_bwd followed by gsr_adam_step (Sec. III-C: visible
 * Gaussians of the latest segments are refined by a sparse gradient optimiser): the parameter
 * gradients never leave registers.  For every Gaussian visible in at least one view (tile_info
 * row 0 > 0) whose segment_id >= min_segment (segment_id NULL = all), the
 * Adam update of gsr_adam_step is applied IN PLACE to the parameter arrays of g, with the moments
 * in adam->m / adam->v (same layouts), per-group learning rates adam->lr = {means, log_scales,
 * quats, opacity_logits, sh rows 0-2 (DC), sh rows 3.. (rest)} and the 1-based step number read
 * from device memory (*adam->step, so a captured graph can replay with an incremented step).
 * All other rows are untouched.  dinst, em, tile_info, dpose and row_mask as in
 * gsr_project_bwd. */
typedef struct {
    gsr_param_grads m, v;
    float lr[6];
    float beta1, beta2, eps;
    const int32_t *step;
} gsr_adam_fused;
GSR_API gsr_status gsr_project_bwd_adam(const gsr_gaussians *g, const gsr_camera *cams, int32_t n_views,
                                        const gsr_raster *r, const gsr_splat *splats, const float *dinst,
                                        const gsr_emission *em, const uint32_t *tile_info,
                                        const uint32_t *visible_list, const uint32_t *visible_count,
                                        const int32_t *segment_id, int32_t min_segment, const gsr_adam_fused *adam,
                                        double *dpose, uint8_t *row_mask, void *ws, size_t ws_bytes,
                                        gsr_stream stream);

/* Ordered list of the Gaussians visible in at least one view (tile_info row 0 > 0 for some
 * view): list [n] receives their indices in ascending order and *count (device) their number.
 * Passing it to gsr_project_bwd_adam (visible_list, visible_count; both or neither) makes the
 * backward launch dense work over the visible Gaussians only; row_mask is then written for the
 * listed rows only.  ws: gsr_visible_list_workspace(n) bytes. */
GSR_API size_t gsr_visible_list_workspace(int64_t n);
GSR_API gsr_status gsr_visible_list(const uint32_t *tile_info, int64_t n, int32_t n_views, uint32_t *list,
                                    uint32_t *count, void *ws, size_t ws_bytes, gsr_stream stream);

/* gsr_visible_list for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same outputs, with no workspace argument.
 * Its block counts live in a fixed device array inside the library (256 KiB, one copy on each GPU
 * it runs on, held until the process ends), so n is limited to gsr_visible_list_noalloc_max()
 * = 16,777,216 Gaussians; larger n returns GSR_E_CAPACITY before anything is launched.  The
 * library allocates and frees nothing here.  The first call on a device looks the array's address
 * up (no allocation); make that first call outside a graph capture.  All calls on one GPU share
 * the array: calls that overlap in time on one GPU (two streams, two threads) race and must be
 * ordered by the caller.  Errors as gsr_visible_list, plus GSR_E_HIP if the look-up fails. */
GSR_API int64_t gsr_visible_list_noalloc_max(void);
GSR_API gsr_status gsr_visible_list_noalloc(const uint32_t *tile_info, int64_t n, int32_t n_views, uint32_t *list,
                                            uint32_t *count, gsr_stream stream);

/* ---- sparse Adam -----------------------------------------------------------------------------
 * Sparse gradient optimiser of Sec. III-C (visible and unfrozen Gaussians only).  Up to 8
 * parameter groups, each a [cols][rows] component-major float32 tensor sharing the row count
 * `rows` (one row per Gaussian).  For rows with row_mask != 0 (row_mask NULL = every row):
 * m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step))
 * + eps).  Masked-out rows keep p, m, v.  Every gradient element is zeroed.  step >= 1. */
#define GSR_MAX_GROUPS 8
typedef struct {
    float *param[GSR_MAX_GROUPS];
    float *grad[GSR_MAX_GROUPS];
    float *m[GSR_MAX_GROUPS];
    float *v[GSR_MAX_GROUPS];
    int32_t cols[GSR_MAX_GROUPS];
    float lr[GSR_MAX_GROUPS];
    int32_t n_groups;
    int32_t _pad;
} gsr_adam_groups;
GSR_API gsr_status gsr_adam_step(const gsr_adam_groups *groups, int64_t rows, const uint8_t *row_mask, float beta1,
                         float beta2, float eps, int32_t step, gsr_stream stream);

/* ---- per-step preparation of the batched optimiser (Sec. III-C: each iteration draws its views
 * from the recent and history keyframe windows; sparse Adam) --------------------------------------
 * One launch for the bookkeeping at the start of an optimisation step:
 * cams [n_views] (device, OVERWRITTEN) = pool[view_idx[v]] (pool: device gsr_camera [n_pool];
 * view_idx: device int64 [n_views], each in [0, n_pool); a record whose index lies outside is
 * left unchanged); view_idx32 [n_views] (device int32, may be NULL) = view_idx, the slot indices
 * the loss kernels read targets with; *loss (device float64, may be NULL) = 0; *step (device
 * int32, may be NULL) += 1, the step number gsr_project_bwd_adam reads; row_mask [n] (device
 * uint8, 16-byte aligned, may be NULL) = 0.
 * Errors: GSR_E_INVALID (a NULL pool, view_idx or cams, n_pool < 1, n_views < 1, n < 0, or an
 * unaligned row_mask). */
GSR_API gsr_status gsr_step_prep(const gsr_camera *pool, int32_t n_pool, const int64_t *view_idx, int32_t n_views,
                                 gsr_camera *cams, int32_t *view_idx32, double *loss, int32_t *step,
                                 uint8_t *row_mask, int64_t n, gsr_stream stream);

/* ---- L1 loss ---------------------------------------------------------------------------------
 * Eq. 9, 10, 12 with lambda_rgb = 1, lambda_ssim = 0 and the all-ones mask, per view v:
 * L_v = (1/P) sum_x sum_ch |C - C~| + lambda_depth (1/P) sum_x |D - D~|, P = W H; the loss is
 * summed over views into *loss (device float64, ACCUMULATED).  Writes dL_drgb [V][3][H][W] and,
 * if dL_ddepth is not NULL, dL_ddepth [V][H][W] (sign(0) = 0).  Targets are read from slot
 * target_index[v] (device int32 [V]; NULL = slot v) of target_rgb [S][3][H][W] and
 * target_depth [S][H][W]; target_depth may be NULL (then lambda_depth is ignored and
 * dL_ddepth, if given, is zeroed). */
GSR_API gsr_status gsr_loss_l1(const float *rgb, const float *depth, const float *target_rgb, const float *target_depth,
                       const int32_t *target_index, int32_t n_views, const gsr_raster *r, float lambda_depth,
                       double *loss, float *dL_drgb, float *dL_ddepth, gsr_stream stream);

/* ---- supervision masks (Sec. III-C, Eq. 7) -------------------------------------------------
 * Geometric support M_geo(x) = [T_final(x) <= 1 - tau_geo] (accumulated opacity at least tau_geo,
 * the comparison taken in float32 against the float32 value 1 - tau_geo), and the interior mask
 * M_int = binary erosion of M_geo by the disk dx^2 + dy^2 <= r_erode^2, pixels outside the image
 * counting as unsupported.  T_final [V][H][W] as written by the forward render.  Writes
 * mask [V][H][W] (uint8, 1 = in M_int) and count [V] (uint32, |M_int| per view, OVERWRITTEN).
 * tau_geo in [0, 1], r_erode in [0, 8], else GSR_E_INVALID. */
GSR_API gsr_status gsr_support_mask(const float *T_final, int32_t n_views, const gsr_raster *r, float tau_geo,
                                    int32_t r_erode, uint8_t *mask, uint32_t *count, gsr_stream stream);

/* ---- full training loss (Sec. III-C, Eq. 9-12) ------------------------------------------------
 * Per view v with mask M (mask NULL = all pixels, count then unused; else count[v] = |M| as from
 * gsr_support_mask):
 *   L_v = lambda_rgb (1/|M|) sum_{x in M} sum_ch |C - C~|            (Eq. 10)
 *       + lambda_ssim (1 - SSIM(M C, M C~))                          (Eq. 11)
 *       + lambda_depth (1/|M|) sum_{x in M} |D - D~|                 (Eq. 12)
 * where SSIM is the mean over the pixels of M and the three channels of the SSIM map of the
 * mask-restricted images (both multiplied by M): 11 x 11 Gaussian window of sigma 1.5, zero
 * padding outside the image, C1 = 0.01^2, C2 = 0.03^2.  A view with an empty mask adds nothing.
 * The loss is summed over views into *loss (device float64, ACCUMULATED); dL_drgb [V][3][H][W]
 * and dL_ddepth [V][H][W] (may be NULL) are OVERWRITTEN (sign(0) = 0; zero off the mask).
 * Targets are read from slot target_index[v] (NULL = slot v) of target_rgb [S][3][H][W] and
 * target_depth [S][H][W] (may be NULL: no depth term).  ws: gsr_loss_workspace(V, r) bytes,
 * 256-byte aligned (the per-pixel SSIM derivative maps and per-block partial sums, which are
 * added in a fixed order, so the loss value is reproducible). */
GSR_API size_t gsr_loss_workspace(int32_t n_views, const gsr_raster *r);
GSR_API gsr_status gsr_loss(const float *rgb, const float *depth, const float *target_rgb, const float *target_depth,
                            const int32_t *target_index, int32_t n_views, const gsr_raster *r, const uint8_t *mask,
                            const uint32_t *count, float lambda_rgb, float lambda_ssim, float lambda_depth,
                            double *loss, float *dL_drgb, float *dL_ddepth, void *ws, size_t ws_bytes,
                            gsr_stream stream);

/* ---- map maintenance (Sec. III-C) -------------------------------------------------------------
 * Low-opacity pruning under a bounded removal ratio.  Candidates are the rows with
 * opacity_logits[i] < max_logit (opacity below sigmoid(max_logit)) and, when segment_id is not
 * NULL, segment_id[i] >= min_segment (frozen segments are never pruned).  At most
 * k = floor((double)max_ratio * n) rows are removed: every candidate when there are at most k,
 * else the k candidates with the smallest logits, equal logits in ascending row order.
 * keep_index [n] receives the surviving rows in ascending order and *n_keep (device uint32)
 * their count; compact the arrays with gsr_gather_rows.  n < 2^32 - 1, max_ratio in [0, 1].
 * ws: gsr_prune_workspace(n) bytes, 256-byte aligned. */
GSR_API size_t gsr_prune_workspace(int64_t n);
GSR_API gsr_status gsr_prune_select(const float *opacity_logits, const int32_t *segment_id, int32_t min_segment,
                                    int64_t n, float max_logit, float max_ratio, uint32_t *keep_index,
                                    uint32_t *n_keep, void *ws, size_t ws_bytes, gsr_stream stream);

/* ---- row order for memory locality -------------------------------------------------------------
 * Not a step of the paper's method: the order in which the map's rows are stored.  The paper's
 * segments grow by appending, and the optimisation updates only the K latest segments (Sec.
 * III-C); keeping rows grouped by segment, and spatially ordered inside a segment, makes the rows
 * one step touches (visible, and in the latest segments) dense in memory.
 * order[j] (uint32 [n], written) = the row that moves to position j: rows sorted by segment_id
 * (int32 [n], ascending; NULL = one segment), then by the Morton code of the mean (means
 * float32 [3][n]) on a 1024^3 grid over the means' bounding box, then by row index.  A
 * coordinate's cell is floor((x - lo) * (1024 / (hi - lo))) evaluated in float32 in that order
 * (0 when hi = lo), clamped to [0, 1023]; the code interleaves the ten bits of the x, y and z
 * cells with x lowest.  Move the rows with gsr_gather_rows(groups, n, order, n, n, 0) into new
 * arrays.  ws: gsr_row_order_workspace(n) bytes, 256-byte aligned.  Errors: GSR_E_INVALID (bad
 * pointers, n >= 2^32), GSR_E_CAPACITY (ws_bytes too small). */
GSR_API size_t gsr_row_order_workspace(int64_t n);
GSR_API gsr_status gsr_row_order(const float *means, const int32_t *segment_id, int64_t n, uint32_t *order,
                                 void *ws, size_t ws_bytes, gsr_stream stream);

/* Row gather over groups of component-major arrays of 4-byte elements (float32 / int32):
 *   dst[g][c * dst_rows + dst_offset + j] = src[g][c * src_rows + r_j],  r_j = index ? index[j] : j
 * for j < n_rows, c < cols[g].  Compaction: index = keep_index, dst_offset = 0; appending rows:
 * two calls into one destination with different offsets.  Requires dst_offset + n_rows <=
 * dst_rows; rows r_j >= src_rows are skipped.  src and dst must not overlap. */
#define GSR_MAX_ROW_GROUPS 16
typedef struct {
    const void *src[GSR_MAX_ROW_GROUPS];
    void *dst[GSR_MAX_ROW_GROUPS];
    int32_t cols[GSR_MAX_ROW_GROUPS];
    int32_t n_groups;
    int32_t _pad;
} gsr_row_groups;
GSR_API gsr_status gsr_gather_rows(const gsr_row_groups *groups, int64_t src_rows, const uint32_t *index,
                                   int64_t n_rows, int64_t dst_rows, int64_t dst_offset, gsr_stream stream);

/* Proximity filter for newly initialised Gaussians (spatial test in 3-D Euclidean space): new
 * mean j is redundant when a map mean lies strictly within d_min, the squared distance taken in
 * float64 from the float32 coordinates as ((dx dx + dy dy) + dz dz) with every operation rounded
 * separately and compared with (double)d_min squared.  Means are [3][n] (coordinates below 10^6 m
 * in magnitude).  Writes keep [n_new] (uint8, 1 = insert), keep_index [n_new] (kept rows,
 * ascending) and *n_keep (device uint32).  d_min > 0; n_map, n_new < 2^32 - 1.
 * ws: gsr_proximity_workspace(n_map, n_new) bytes, 256-byte aligned. */
GSR_API size_t gsr_proximity_workspace(int64_t n_map, int64_t n_new);
GSR_API gsr_status gsr_proximity_filter(const float *map_means, int64_t n_map, const float *new_means, int64_t n_new,
                                        float d_min, uint8_t *keep, uint32_t *keep_index, uint32_t *n_keep, void *ws,
                                        size_t ws_bytes, gsr_stream stream);

/* ---- Gaussian-based loop registration (Sec. III-D, Eq. 13-16) -------------------------------------
 * Geometric decisions are taken in float64 from the float32 inputs with every operation rounded
 * separately, in this order: camera k sees mean mu when, with p = R mu + t computed per coordinate
 * as ((R_r0 x + R_r1 y) + R_r2 z) + t_r, z > z_near and u = fx (x / z) + cx in [0, W),
 * v = fy (y / z) + cy in [0, H); its centre is c = -R^T t (each coordinate
 * -((R_0i t_0 + R_1i t_1) + R_2i t_2)); squared distances are ((dx dx + dy dy) + dz dz).
 *
 * gsr_gicp_prepare: the source set (rows with segment_id == src_segment) into src_index and the
 * target set of Eq. 13 (rows outside the source set that some camera of cams [n_cams] (device)
 * sees, with the camera centre closer than d_max) into tgt_index, both in ascending row order,
 * counts (device uint32 [2]) = (n_src, n_tgt).  Every listed Gaussian's covariance R_q S^2 R_q^T
 * has its eigenvalues replaced by (1, 1, 1e-3), the 1e-3 on the smallest-scale axis (the first
 * on ties), and the target means are gridded for d_corr; all of it is kept in ws.  stats (device
 * double [40]) is cleared.  g supplies means, log_scales and quats; src_index, tgt_index [n].
 *
 * gsr_gicp_iterate: n_iter Gauss-Newton iterations of Eq. 16 from pose (device double [12]: R
 * row-major, then t; the transform applied to the source means), updated in place.  Each
 * iteration pairs source mean m, moved to q = R mu_m + t, with the nearest target mean strictly
 * within d_corr (lowest target position on ties), forms r = mu_n - q, C = S_n + R S_m R^T,
 * W = C^-1, J = dr/dxi = [-I, [q]x] for the left perturbation xi = (rho, phi), sums
 * H = J^T W J, g = J^T W r, cost = r^T W r, |r|^2 and the count, solves H xi = -g and sets
 * (R, t) <- (Exp(phi) R, Exp(phi) t + rho).  stats: [0, 21) H upper triangle row-major, [21, 27) g,
 * 27 cost, 28 sum |r|^2, 29 count (of the last linearisation), [30, 36) the last xi, 36 converged
 * (last step |rho| < 2.5e-3 m and |phi| < 2.5e-4 rad), 37 iterations done, 38 failed (fewer than 6 correspondences
 * or H not positive definite).  Once converged or failed, further iterations do nothing.  corr
 * (device int32 [n], may be NULL) receives, per source position, the target position of the last
 * linearisation or -1.  Call with the same g, index arrays, d_corr and ws as gsr_gicp_prepare.
 * ws: gsr_gicp_workspace(n) bytes, 256-byte aligned.  d_max, d_corr > 0. */
GSR_API size_t gsr_gicp_workspace(int64_t n);
GSR_API gsr_status gsr_gicp_prepare(const gsr_gaussians *g, const int32_t *segment_id, int32_t src_segment,
                                    const gsr_camera *cams, int32_t n_cams, float d_max, float d_corr,
                                    uint32_t *src_index, uint32_t *tgt_index, uint32_t *counts, double *stats,
                                    void *ws, size_t ws_bytes, gsr_stream stream);
GSR_API gsr_status gsr_gicp_iterate(const gsr_gaussians *g, const uint32_t *src_index, const uint32_t *tgt_index,
                                    const uint32_t *counts, float d_corr, double *pose, double *stats, int32_t *corr,
                                    int32_t n_iter, void *ws, size_t ws_bytes, gsr_stream stream);

/* ---- voxel-PCA geometric fitting (Sec. III-A, Eq. 1-2) ------------------------------------------
 * Points [3][n] (float32, world frame) are binned into 0.5 m voxels, key floor(p / 0.5), valid for
 * x, y in [-512, 512) m and z in [-255.5, 256) m (points outside are counted in *n_outside and
 * belong to no voxel).  Voxels are numbered in ascending (kx, ky, kz) order.  Inside a voxel the
 * points are ordered by ascending SplitMix64(seed XOR point index); the first min(count, 32) are
 * the voxel's fitting points.  Per voxel (arrays sized n, component-major with stride n):
 * mean and biased covariance of the fitting points, eigenvalues ascending, R_pca (row-major, columns
 * v_max, v_mid, v_min, each with its largest-magnitude component positive, then v_min flipped so
 * that det = +1), s_pca = 0.5 log max(lambda, (5 mm)^2) per column, class (planar if
 * lambda_min < 2.5e-3 m^2, else linear if lambda_max / lambda_min > 4, else unreliable; also
 * unreliable below 5 points), the trace of the direction block of the descriptor covariance
 * (Eq. 1-2 with every point covariance (2 cm)^2 I) and reliable = (planar or linear) and
 * trace < 0.1^2.  ws: gsr_voxel_pca_workspace(n) bytes, 256-byte aligned. */
typedef struct {
    uint32_t *n_voxels;    /* [1] */
    uint32_t *n_outside;   /* [1] */
    uint32_t *key;         /* [n] packed (kx+1024) << 21 | (ky+1024) << 10 | (kz+511), ascending */
    uint32_t *start;       /* [n] first entry of the voxel in point_order */
    uint32_t *count;       /* [n] points in the voxel */
    uint32_t *point_order; /* [n] point indices grouped by voxel, hash order inside */
    uint32_t *point_voxel; /* [n] voxel of each point, 0xffffffff outside the key range */
    float *mu;             /* [3][n] */
    float *evals;          /* [3][n] ascending */
    float *R;              /* [9][n] row-major R_pca */
    float *s_pca;          /* [3][n] */
    float *trace;          /* [n] (infinity when unreliable by class) */
    uint8_t *cls;          /* [n] 0 planar, 1 linear, 2 unreliable */
    uint8_t *reliable;     /* [n] */
} gsr_voxels;
GSR_API size_t gsr_voxel_pca_workspace(int64_t n);
GSR_API gsr_status gsr_voxel_pca(const float *points, int64_t n, uint64_t seed, const gsr_voxels *out, void *ws,
                                 size_t ws_bytes, gsr_stream stream);
/* As gsr_voxel_pca with each point's world-frame covariance Sigma_i^W (point_cov [6][n] =
 * xx, xy, xz, yy, yz, zz; measurement and pose noise) in Eq. 2: for a planar or linear voxel,
 * Sigma_g = sum_i J_i Sigma_i J_i^T over its fitting points with J_i = [V F_i; I/N] of Eq. 1
 * (V = [v_min v_mid v_max], the R_pca columns in reverse; f_i^(m) = (p_i - mu)^T (v_m v_k^T +
 * v_k v_m^T) / (N (lambda_k - lambda_m)) for m != k, k = min for planar and max for linear).
 * trace and reliable come from its direction block; sigma_g [21][n] (may be NULL) receives the
 * upper triangle of Sigma_g row-major per voxel (zero for unreliable-class voxels). */
GSR_API gsr_status gsr_voxel_pca_cov(const float *points, const float *point_cov, int64_t n, uint64_t seed,
                                     const gsr_voxels *out, float *sigma_g, void *ws, size_t ws_bytes,
                                     gsr_stream stream);

/* ---- cascaded initialisation (Sec. III-B, Eq. 3, 5, 6) ----------------------------------------
 * One Gaussian per point: mean = point, SH DC = (colour - 0.5) / Y_00, higher SH = 0, and by Eq. 3
 *   model branch      if the point's voxel has a valid prediction (pred [8][n] per voxel, stride
 *                     n: log-scales s[3], quaternion q[4], opacity logit; valid = finite, q != 0,
 *                     s in [log 2 mm, log 0.5 m]): s, q / |q|, logit taken from it;
 *   PCA branch        else if the voxel is reliable: q from R_pca, s = s_pca + log beta (Eq. 5);
 *   heuristic branch  else: q = identity, s = log(depth / focal) on every axis (Eq. 6);
 * non-model branches get opacity 0.1.  beta > 0 is used as given; otherwise per segment
 * beta = clamp(1 - rho, 0.5, 1), rho = the fraction of the segment's points that are reliable
 * but lack a valid prediction (segment [n] int32 in [0, n_segments), NULL = one segment).
 * pred may be NULL (no model).  Outputs: the parameter arrays of out ([c][n]) and branch [n]
 * (0 model, 1 PCA, 2 heuristic).  ws: gsr_cascade_workspace(n_segments) bytes. */
typedef struct {
    float *means, *log_scales, *quats, *opacity_logits, *sh;
} gsr_params;
GSR_API size_t gsr_cascade_workspace(int32_t n_segments);
GSR_API gsr_status gsr_cascade(const float *points, const float *colors, const float *depth, const int32_t *segment,
                               int32_t n_segments, int64_t n, const gsr_voxels *vox, const float *pred, float focal,
                               float beta, int32_t sh_degree, const gsr_params *out, uint8_t *branch, void *ws,
                               size_t ws_bytes, gsr_stream stream);
/* As gsr_cascade with the model branch of Eq. 4: the prediction's log-scales are read as an axis
 * ratio only, a = exp(s - max(s)), and anchored at the point's depth, s_out = log((d / focal) a),
 * so an isotropic prediction gives the heuristic branch's size (the validity test is unchanged). */
GSR_API gsr_status gsr_cascade_anchored(const float *points, const float *colors, const float *depth,
                                        const int32_t *segment, int32_t n_segments, int64_t n, const gsr_voxels *vox,
                                        const float *pred, float focal, float beta, int32_t sh_degree,
                                        const gsr_params *out, uint8_t *branch, void *ws, size_t ws_bytes,
                                        gsr_stream stream);

/* ---- training targets of the model branch (Sec. III-B) ------------------------------------------
 * The point network learns what the plain optimiser makes of the Gaussians a voxel's points seed.
 * For every voxel v of gsr_voxel_pca (arrays sized n, stride n): over ALL the voxel's points i (one
 * Gaussian per point, row i of gauss: log_scales [3][n], quats [4][n] raw (w, x, y, z),
 * opacity_logits [n]; means and sh are not read), the mean covariance
 * R(q_i / |q_i|) diag(exp(2 s_i)) R^T as cov_t [6][n] (xx, xy, xz, yy, yz, zz) and the mean opacity
 * 1 / (1 + exp(-logit_i)) as o_t [n]; has [n] = 1 for a voxel with points, 0 (and zero targets)
 * for rows at or past the voxel count.  Sums in float64 in the voxel's point order (fixed), so the
 * targets repeat exactly.  Errors: GSR_E_INVALID for bad sizes or NULL pointers. */
GSR_API gsr_status gsr_voxel_targets(const gsr_params *gauss, int64_t n, const gsr_voxels *vox, float *cov_t,
                                     float *o_t, uint8_t *has, gsr_stream stream);

/* ---- point network of the model branch (Sec. III-B, Eq. 3) ------------------------------------
 * Per voxel of gsr_voxel_pca: 32 input rows (the fitting points repeated cyclically, centred on the
 * voxel mean, divided by 0.5 m) -> shared MLP 3 -> 64 -> 64 -> 64 with ReLU -> max over the rows
 * -> concat 12 features (log(max(lambda, (5 mm)^2) / 0.25) ascending, then v_min, v_mid, v_max)
 * -> 76 -> 64 with ReLU -> 64 -> 8 = (log-scales[3], quaternion[4], opacity logit), the prediction
 * gsr_cascade reads.  BF16 rounding (nearest even) of the weights and of every GEMM input, FP32
 * bias, ReLU and accumulation; the two 64 x 64 layers run on the matrix cores.  weights: the
 * float32 flat layout W1[3][64] b1[64] W2[64][64] b2 W3[64][64] b3 W4[76][64] b4 W5[64][8] b5[8]
 * (gsr_pointnet_weight_count() floats).  y: [8][n] (stride n, like the voxel arrays). */
GSR_API int gsr_pointnet_weight_count(void);
GSR_API gsr_status gsr_pointnet_fwd(const float *points, int64_t n, const gsr_voxels *vox, const float *weights,
                                    float *y, gsr_stream stream);
/* Gradient of the training loss with respect to the weights, OVERWRITTEN into grad (flat layout):
 * the sum over voxels with a target (tmask [n] nonzero; NULL = all) of inv_count times
 * KL(N(0, Sigma_pred) || N(0, Sigma_tgt)) + 0.1 |sigmoid(omega) - o_tgt|, with
 * Sigma_pred = R(q / |q|) diag(exp(2 s)) R(q / |q|)^T, targets cov_t [6][n] = (xx, xy, xz, yy, yz, zz)
 * and o_t [n].  The backward GEMMs round their inputs (upstream gradients included) to BF16; the
 * max-pool routes to the argmax row (lowest row on ties).  The loss value is ADDED to *loss
 * (device float64).  blocks: persistent workgroups (each keeps partial sums, reduced in a fixed
 * order); ws: gsr_pointnet_bwd_workspace(blocks) bytes. */
GSR_API size_t gsr_pointnet_bwd_workspace(int32_t blocks);
GSR_API gsr_status gsr_pointnet_bwd(const float *points, int64_t n, const gsr_voxels *vox, const float *weights,
                                    const float *cov_t, const float *o_t, const uint8_t *tmask, float inv_count,
                                    int32_t blocks, float *grad, double *loss, void *ws, size_t ws_bytes,
                                    gsr_stream stream);

/* ---- propagation of a corrected pose to a segment (Sec. III-D) ----------------------------------
 * The Gaussians with segment_id == segment move rigidly by pose (device double [12]: R row-major,
 * then t; world -> world): means R mu + t, quaternions q_R (x) q with q_R the unit quaternion of R
 * (w >= 0; the raw quaternion's norm is kept), and every SH degree l >= 1 of every colour channel
 * c' = D_l c with D_ab = the integral over the sphere of Y_a(d) Y_b(R^T d), so that the colour seen
 * along R d afterwards equals the colour seen along d before.  Arithmetic in float64, stored as
 * float32; p->means, p->quats and p->sh are updated in place (log-scales and opacities unchanged).
 * ws: device double [96], scratch for D_1..D_3 and q_R.  gsr_transform_cameras moves the cameras
 * flagged in mask [n_cams] (device uint8; NULL = all) of a device array with the same transform:
 * world -> camera (R_c, t_c) becomes (R_c R^T, t_c - R_c R^T t). */
GSR_API gsr_status gsr_transform_segment(const gsr_params *p, int64_t n, int32_t sh_degree, const int32_t *segment_id,
                                         int32_t segment, const double *pose, double *ws, gsr_stream stream);
GSR_API gsr_status gsr_transform_cameras(gsr_camera *cams, int32_t n_cams, const uint8_t *mask, const double *pose,
                                         gsr_stream stream);

/* Fill n 32-bit words with a value (graph-capture safe replacement for memset). */
GSR_API gsr_status gsr_fill_u32(void *dst, uint32_t value, int64_t n_words, gsr_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* GSR_H */
