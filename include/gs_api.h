/*
 * gs_api.h -- C ABI of the MI355X (gfx950) differentiable Gaussian-splatting
 * rasterizer that every joint camera-pose / Gaussian optimisation step runs
 * forward and backward (paper section 4.3: 30 such iterations per keyframe,
 * sparse Adam on the Gaussians, poses optimised jointly and receiving
 * gradient through Gaussian position and rotation but not through the
 * spherical harmonics), plus the primitive-spawning step of section 4.2,
 * the multi-scale training helpers of section 4.3 (screen-space filter,
 * coarse-to-fine pyramid, per-Gaussian learning rates, opacity culling),
 * the guided-matching depth of new primitives, the anchor decisions of
 * section 4.4 (creation trigger, two-anchor blending), and measurement
 * probes.
 *
 * The rasterizer is the EWA splatting model of the 3DGS codebase the paper
 * builds on (section 5): Gaussians with mean, log-scales, rotation
 * quaternion, opacity logit and SH colour are projected to 2D Gaussians, and
 * every pixel composites them front to back in depth order until its
 * transmittance would fall below a cutoff.
 *
 * Conventions that hold for every entry point:
 *   * Memory.  Every array argument is caller-owned DEVICE memory unless it is
 *     marked "host".  The library never allocates device memory; scratch
 *     comes in through workspace arguments whose sizes the *_workspace
 *     queries return.  Arrays are float32 structure-of-arrays planes: a
 *     parameter with k components over n Gaussians is k contiguous planes of
 *     n values ("[k][n]").
 *   * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Every
 *     call is asynchronous on it, except where a call says it synchronises.
 *   * Errors.  Arguments are checked on the host before anything is
 *     launched; a failed check launches nothing and returns
 *     GS_ERR_INVALID_ARG.  A failed HIP call returns GS_ERR_HIP.
 *     gs_last_error() returns a thread-local text for the last non-OK status.
 *     No C++ exception crosses the ABI.
 *   * Non-finite values.  A Gaussian whose projection is not finite (a NaN
 *     or infinite mean, scale, rotation or opacity, or a 2D covariance
 *     whose inverse overflows) is culled by the projection: it touches no
 *     tile, composites nothing and receives zero gradient.  A NaN or
 *     infinite SH coefficient of a visible Gaussian is not detected in
 *     normal operation and reaches the image.  With GS_CHECK_FINITE set
 *     (to anything but "0") in the environment, gs_project(_views) count
 *     the non-finite values of the Gaussians and poses, gs_render_fwd(_l1)
 *     those of the image and depth they write, and gs_render_bwd those of
 *     the upstream gradients and of the gradients it accumulates; any
 *     count above 0 returns GS_ERR_NONFINITE (gs_last_error names the
 *     array and the count).  The checks synchronise the stream, share one
 *     8-byte device counter per GPU held by the library, and are
 *     serialised by a host lock.
 *   * Gradients accumulate (+=) into caller buffers, so several views can
 *     be summed; the caller zeroes them.
 *   * Camera.  World->camera pose [R | t] with R row-major; the camera looks
 *     down +z; pixel (u, v) is sampled at the continuous point (u, v); the
 *     projected mean is (fx x/z + cx, fy y/z + cy).
 *   * Thread safety.  Entry points may be called from several host threads
 *     on different streams, except the profiling switches.
 */
#ifndef GS_API_H
#define GS_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GS_OK = 0,
  GS_ERR_INVALID_ARG = 1, /* bad pointer, size, degree, ...; nothing launched */
  GS_ERR_CAPACITY = 2,    /* an output is too small; the required size is returned */
  GS_ERR_HIP = 3,         /* a HIP runtime call failed */
  GS_ERR_WORKSPACE = 4,   /* the workspace is smaller than the query returned */
  GS_ERR_NONFINITE = 5    /* debug mode only (GS_CHECK_FINITE=1): a NaN or an infinity
                             in an input, or produced in an output; see below */
} gs_status;

/* Tile edge in pixels; the render kernels map one 16x16 tile to one
 * 256-lane workgroup (four wave64). */
#define GS_TILE 16

/* Render record written by gs_project, one per Gaussian, 16 floats (64 B,
 * half a 128-byte cache line, so a gather touches one line):
 *   [0] mean_x integer part   [1] mean_y integer part   (exact integers)
 *   [2] mean_x - [0]          [3] mean_y - [1]          (in [-0.5, 0.5])
 *   [4] A  [5] B  [6] C       conic: inverse 2D covariance [[A, B], [B, C]]
 *   [7] opacity o = sigmoid(logit)
 *   [8] [9] [10] colour (r, g, b) from SH, clamped below at 0
 *   [11] depth z of the camera-space mean (positive)
 *   [12] [13] half-extents (hx, hy) in pixels of the bounding box of the
 *        support ellipse d^T conic d <= 2 ln(o / alpha_min)
 *   [14] [15] zero
 * The split mean keeps the offset to a pixel exact to ~1e-7 px at any image
 * size.  The FP32 mean used for binning is the sum of the two parts rounded
 * once: mean_x = fl(rec[0] + rec[2]), mean_y = fl(rec[1] + rec[3]). */
#define GS_REC_FLOATS 16

typedef struct {
  int32_t width, height;    /* image size in pixels, 1 .. 16384 */
  float fx, fy, cx, cy;     /* pinhole intrinsics in pixels, fx, fy > 0 */
  float near_plane;         /* Gaussians with camera depth <= near are culled */
  float bg[3];              /* background colour composited behind everything */
  const float *pose;        /* DEVICE [12]: R (row-major 3x3) then t (3), world->camera */
} gs_camera;                /* passed by pointer to HOST memory */

typedef struct {
  float eps2d;     /* dilation added to the 2D covariance's diagonal (0.3) */
  float alpha_max; /* opacity clamp of a single Gaussian at a pixel (0.99) */
  float alpha_min; /* smaller alphas are skipped (1/255) */
  float t_min;     /* a pixel stops before transmittance would drop below this (1e-4) */
  float guard;     /* guard band of the perspective Jacobian, in half-FOVs (1.3) */
  int32_t mip_filter; /* 0: eps2d is the 3DGS dilation; else the screen-space filter
                         of multi-scale training (section 4.3, Mip-Splatting): eps2d
                         is the filter's variance (0.1 there) and each splat's opacity
                         is scaled by sqrt(det Sigma2_raw / det Sigma2) (default 0) */
} gs_raster_params;  /* HOST memory */

typedef struct {
  int64_t n;          /* number of Gaussians, 0 .. 2^31 - 1 */
  int32_t sh_degree;  /* 0 .. 3 */
  float *means;          /* [3][n] world-space mean */
  float *log_scales;     /* [3][n] log of the per-axis standard deviation */
  float *quats;          /* [4][n] rotation (w, x, y, z), normalised inside */
  float *opacity_logits; /* [n]    opacity = sigmoid(logit) */
  float *sh;             /* [(deg+1)^2][3][n] SH coefficients per colour channel */
  float *filter3d;       /* [n] or NULL: variance v of the 3D smoothing filter of
                            multi-scale training (section 4.3, Mip-Splatting): the
                            projection uses axis variances s^2 + v in the same
                            rotation and opacity o prod s / sqrt(s^2 + v) (the
                            Gaussian convolved with an isotropic low-pass, its
                            integral kept); gradients flow to the log-scales and
                            the logit, none to v.  Read by the projection and its
                            adjoint only; ignored in gradient structs. */
} gs_gaussians;          /* HOST struct of DEVICE pointers */

typedef struct {
  float *rec;             /* [n][GS_REC_FLOATS] render records (layout above) */
  int32_t *radius;        /* [2][n] integer half-widths (rx, ry) of the support rect, rx = 0: culled */
  int32_t *tiles_touched; /* [n] number of 16x16 tiles the support square meets */
  uint32_t *bin;          /* [n][4] or NULL: the binning's inputs, written by the projection
                             where tiles_touched > 0 (elsewhere left as they were): the bits
                             of the depth rec[11], the tile rect as tx0 | ty0 << 16 and
                             tx1 | ty1 << 16 (inclusive, the tiles counted in
                             tiles_touched), 0.  gs_bin_sort(_async) read them when bin is
                             not NULL instead of the records' lines (one 16-byte read per
                             visible Gaussian instead of a 64-byte line and the radii);
                             the lists are the same either way. */
} gs_projected;           /* HOST struct of DEVICE pointers */

/* Fills *p with the constants above (0.3, 0.99, 1/255, 1e-4, 1.3, 0). */
void gs_default_params(gs_raster_params *p);

const char *gs_last_error(void);

/* ---- gs_project ---------------------------------------------------------
 * Per-Gaussian EWA projection (the rasterizer of section 5 / 3DGS):
 *   p = R mean + t; culled if p_z <= near;
 *   J = perspective Jacobian at p, with x/z and y/z clamped to +-guard
 *       half-FOVs (guard band);
 *   Sigma = Rq diag(exp(2 log_scales)) Rq^T, Rq from the normalised quaternion;
 *   Sigma2 = J R Sigma R^T J^T + eps2d I; conic = Sigma2^-1;
 *   colour = max(0, sum_k sh_k Y_k(dir) + 0.5), dir = unit(mean - camera
 *   centre), real SH up to degree 3;
 *   o = sigmoid(logit), times rho = sqrt(det Sigma2_raw / det Sigma2) with
 *   Sigma2_raw = Sigma2 - eps2d I if mip_filter (the splat keeps its
 *   integral o 2 pi sqrt(det Sigma2)); culled if o < alpha_min;
 *   support: the ellipse where o exp(-d^T conic d / 2) >= alpha_min, i.e.
 *   d^T conic d <= qmax = 2 ln(o / alpha_min); its bounding box has
 *   half-extents hx = sqrt(qmax Sigma2_xx), hy = sqrt(qmax Sigma2_yy) and
 *   rx = ceil(hx (1 + 1e-4) + 1e-3), ry likewise; tiles_touched counts the
 *   tiles holding an integer pixel of the clipped rect
 *   [mean_x - rx, mean_x + rx] x [mean_y - ry, mean_y + ry].
 * Geometry is evaluated in FP64 and stored in FP32.  Culled Gaussians get
 * radius = tiles_touched = 0 and zeroed records.
 * Errors: GS_ERR_INVALID_ARG for NULL pointers (n > 0), n < 0, degree out of
 * range, non-positive sizes or focal lengths. */
gs_status gs_project(const gs_camera *cam, const gs_raster_params *rp, const gs_gaussians *g, gs_projected *out,
                     void *stream);

/* ---- gs_bin_sort --------------------------------------------------------
 * Builds the per-tile depth-ordered lists: every (Gaussian, tile) pair of
 * gs_project's support rects, ordered by tile id (row-major tiles,
 * tiles_x = ceil(W/16)), then by the FP32 depth, then by Gaussian index.
 * That is the order of a stable sort of the key (tile << 32 | bits(depth))
 * over pairs emitted in Gaussian-index order.  Implemented as a stable LSD
 * radix sort of the visible Gaussians by depth followed by a stable LSD
 * radix sort of the emitted pairs by tile.
 *   tile_ids   [capacity] out: tile id of each sorted pair
 *   values     [capacity] out: Gaussian index of each sorted pair
 *   slots      [capacity] out: slot of each sorted pair, a bijection onto
 *                         [0, M) numbered by Gaussian index then row-major
 *                         tile of its rect: the pairs of Gaussian g have
 *                         slots first_slot[g] .. first_slot[g] +
 *                         tiles_touched[g] - 1, first_slot being the
 *                         exclusive prefix sum of tiles_touched
 *   ranges     [T][2]     out: [start, end) of each tile's run (0,0 if empty)
 *   first_slot [n]        out: first slot of each Gaussian (written where
 *                         tiles_touched > 0)
 *   n_instances (HOST)    out: the number M of pairs
 * Synchronises the stream once (4-byte read of M).  If M > capacity it
 * returns GS_ERR_CAPACITY with *n_instances = M and writes no list output.
 * ws must be at least gs_bin_sort_workspace(n, capacity) bytes. */
gs_status gs_bin_sort_workspace(int64_t n, int64_t capacity, size_t *bytes);
gs_status gs_bin_sort(const gs_camera *cam, const gs_projected *proj, int64_t n, int64_t capacity, void *ws,
                      size_t ws_bytes, uint32_t *tile_ids, uint32_t *values, uint32_t *slots, uint32_t *ranges,
                      uint32_t *first_slot, int64_t *n_instances, void *stream);

/* The same without any host synchronisation: the pair count M goes to
 * *n_instances_dev (DEVICE uint32) and every later kernel reads it there.
 * If M > capacity the lists hold an unspecified subset of the pairs (every
 * index stays below capacity; a Gaussian whose pairs do not all fit gets
 * first_slot 0xffffffff and no gradient) and *n_instances_dev still reports
 * M: the caller checks it (whenever it next synchronises) and repeats the
 * work with more capacity.  For loops whose
 * pair counts are known to fit, e.g. the iterations of an optimisation
 * after the first. */
gs_status gs_bin_sort_async(const gs_camera *cam, const gs_projected *proj, int64_t n, int64_t capacity, void *ws,
                            size_t ws_bytes, uint32_t *tile_ids, uint32_t *values, uint32_t *slots,
                            uint32_t *ranges, uint32_t *first_slot, uint32_t *n_instances_dev, void *stream);


/* ---- gs_render_fwd ------------------------------------------------------
 * Front-to-back compositing per pixel over its tile's list: with
 * d = pixel - mean, alpha = min(alpha_max, o exp(-d^T conic d / 2));
 * alpha < alpha_min is skipped; if T (1 - alpha) < t_min the pixel stops
 * without this Gaussian; otherwise C += colour alpha T, D += z alpha T,
 * T *= 1 - alpha.  Outputs, all [H][W] planes (image [3][H][W]):
 *   image = C + T bg, depth = D (not normalised), alpha = 1 - T,
 *   final_t = T, n_contrib = list entries up to and including the last one
 *   composited (counted from the tile's start; state for the backward),
 *   stats [4][H][W] (NULL = not written), per pixel: plane 0 the tile-list
 *   entries up to and including the one that stopped the pixel (the whole
 *   list if it did not stop), plane 1 the entries evaluated (after culling
 *   entries whose support box misses the pixel's 4x4 sub-block), plane 2 the
 *   entries with alpha >= alpha_min up to and including the stopping one,
 *   plane 3 the entries composited -- the pair counts the work is measured
 *   in.
 * values / ranges from gs_bin_sort. */
gs_status gs_render_fwd(const gs_camera *cam, const gs_raster_params *rp, const gs_projected *proj,
                        const uint32_t *values, const uint32_t *ranges, float *image, float *depth, float *alpha,
                        float *final_t, int32_t *n_contrib, int32_t *stats, void *stream);

/* gs_render_fwd with the L1 photometric loss of the joint optimisation
 * (section 4.3) formed in the same kernel while each pixel's colour is in
 * registers: writes everything gs_render_fwd writes (no stats) and what
 * gs_loss_l1(image, target, grad_scale) writes -- dL_dimage = grad_scale *
 * sign(image - target) with exact zeros, bit-identical to gs_loss_l1's, and
 * sums[0] = sum |image - target|, sums[1] = sum (image - target)^2 (DEVICE
 * double[2], overwritten; summed per tile in FP64, then over the tiles in a
 * fixed order, so they equal gs_loss_l1's up to FP64 rounding).
 * target, dL_dimage: DEVICE [3][H][W].  ws: DEVICE scratch of
 * gs_render_fwd_l1_workspace(width, height) bytes (16 per tile). */
gs_status gs_render_fwd_l1_workspace(int32_t width, int32_t height, size_t *bytes);
gs_status gs_render_fwd_l1(const gs_camera *cam, const gs_raster_params *rp, const gs_projected *proj,
                           const uint32_t *values, const uint32_t *ranges, float *image, float *depth, float *alpha,
                           float *final_t, int32_t *n_contrib, const float *target, float grad_scale,
                           float *dL_dimage, double *sums, void *ws, size_t ws_bytes, void *stream);

/* gs_render_fwd_l1 without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and outputs as
 * gs_render_fwd_l1 minus ws / ws_bytes; allocates nothing: the per-tile loss
 * partials live in a fixed 1 MiB scratch array of the library, one per GPU,
 * held until the process ends.  Images of more than 65,536 tiles (e.g.
 * larger than 4096 x 4096) return GS_ERR_INVALID_ARG.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (on different
 * streams, or from several host threads) race on it and must be serialised
 * by the caller.  Every tile writes its partials before they are read, so
 * nothing carries over from an earlier call. */
gs_status gs_render_fwd_l1_noalloc(const gs_camera *cam, const gs_raster_params *rp, const gs_projected *proj,
                                   const uint32_t *values, const uint32_t *ranges, float *image, float *depth,
                                   float *alpha, float *final_t, int32_t *n_contrib, const float *target,
                                   float grad_scale, float *dL_dimage, double *sums, void *stream);

/* ---- gs_render_bwd ------------------------------------------------------
 * Adjoint of gs_project + gs_render_fwd for upstream gradients of image
 * [3][H][W], depth [H][W] and alpha [H][W] (dL_ddepth / dL_dalpha may be
 * NULL = zero).  image, depth, final_t and n_contrib must be the forward's
 * outputs and values / slots / ranges / first_slot / n_instances
 * gs_bin_sort's for the same inputs.  Accumulates into grads (same layout
 * as g; grads->n and sh_degree must match g) and, if not NULL, into
 *   dL_dpose  [12] (double) gradient w.r.t. R (row-major) and t,
 *   dL_dtwist [6]  (double) gradient w.r.t. a left twist (rho, phi):
 *                  T <- exp(xi^) T, rho the translation part.
 * The pose gradient flows through the projected mean, depth and covariance
 * only, not through the SH view direction (section 4.3).  The Gaussian
 * gradients include the view-direction path.  Decisions (skip, stop, alpha
 * clamp, colour clamp, guard band) are held fixed: the clamp's derivative
 * is zero.  Per-tile contributions go to a per-pair buffer in the workspace
 * (no global atomics) and are summed per Gaussian in slot order.
 * With n_instances == 0 no pixel depends on any Gaussian: the call adds
 * nothing, and values / slots / first_slot may then be NULL.
 * ws: gs_render_bwd_workspace(n, n_instances) bytes. */
gs_status gs_render_bwd_workspace(int64_t n, int64_t n_instances, size_t *bytes);
gs_status gs_render_bwd(const gs_camera *cam, const gs_raster_params *rp, const gs_gaussians *g,
                        const gs_projected *proj, const uint32_t *values, const uint32_t *slots,
                        const uint32_t *ranges, const uint32_t *first_slot, int64_t n_instances, const float *image,
                        const float *depth, const float *final_t, const int32_t *n_contrib, const float *dL_dimage,
                        const float *dL_ddepth, const float *dL_dalpha, gs_gaussians *grads, double *dL_dpose,
                        double *dL_dtwist, void *ws, size_t ws_bytes, void *stream);

/* ---- several views of one window --------------------------------------
 * The joint step renders the same Gaussians from every keyframe of the
 * window (section 4.3).  The projection and its adjoint are bounded by the
 * HBM traffic of the per-Gaussian parameters and gradients, so these forms
 * take a list of views and read each Gaussian's parameters once and write
 * its gradients once per call (up to eight views per pass; longer lists run
 * in passes of eight).  Results equal those of the single-view calls:
 * gs_project_views writes each view's gs_projected exactly as gs_project;
 * gs_render_bwd_pairs + gs_project_bwd_views over one view is gs_render_bwd.
 */
typedef struct {
  gs_camera cam;               /* the view's camera (pose on the device) */
  gs_projected proj;           /* its projection: written by gs_project_views, read by the adjoint */
  const float *pair_grad;      /* DEVICE [M][12] per-pair 2D gradients from gs_render_bwd_pairs */
  const uint32_t *first_slot;  /* DEVICE [n] from gs_bin_sort of this view */
  double *dL_dpose;            /* DEVICE [12] or NULL, accumulated (as gs_render_bwd) */
  double *dL_dtwist;           /* DEVICE [6] or NULL, accumulated */
} gs_view;                     /* HOST array of n_views */

gs_status gs_project_views(int32_t n_views, const gs_view *views, const gs_raster_params *rp,
                           const gs_gaussians *g, void *stream);

/* The compositing adjoint of one view only: writes, for every (Gaussian,
 * tile) pair of the view's lists, its 2D gradient record (dL/d mean x, y,
 * conic A, B, C, opacity, colour r, g, b, depth, 0, 0) into pair_grad
 * [n_instances][12] at the pair's emission slot; arguments as gs_render_bwd.
 * The colour entries are taken through the clamp of the colour at 0 (the
 * colour is max(SH value, 0)): 0 for a channel whose projected colour is
 * not above 0, so the projection adjoint needs no colour record. */
gs_status gs_render_bwd_pairs(const gs_camera *cam, const gs_raster_params *rp, const gs_projected *proj,
                              const uint32_t *values, const uint32_t *slots, const uint32_t *ranges,
                              int64_t n_instances, const float *image, const float *depth, const float *final_t,
                              const int32_t *n_contrib, const float *dL_dimage, const float *dL_ddepth,
                              const float *dL_dalpha, float *pair_grad, void *stream);

/* The projection adjoint over n_views views: per Gaussian, the 2D gradients
 * of its pairs in each view are chained to its parameters and summed over
 * the views into grads (accumulated), and each view's pose gradient goes to
 * its dL_dpose / dL_dtwist.  Runs as two passes per eight views (geometry,
 * then SH).  ws: gs_project_bwd_views_workspace(n, n_views) bytes of DEVICE
 * scratch (FP64 pose partials per workgroup, and each view's clamped colour
 * gradient, 12 bytes per Gaussian, handed from the first pass to the
 * second); its contents are not kept between calls. */
gs_status gs_project_bwd_views_workspace(int64_t n, int32_t n_views, size_t *bytes);
gs_status gs_project_bwd_views(int32_t n_views, const gs_view *views, const gs_raster_params *rp,
                               const gs_gaussians *g, gs_gaussians *grads, void *ws, size_t ws_bytes, void *stream);
/* The same adjoint, but grads receive the sum over the views by plain
 * stores: every Gaussian's gradients are overwritten (0 for one no view
 * saw), so the caller need not clear them first -- one pass over the
 * gradient planes instead of a clearing pass plus a read-modify-write
 * (the pose outputs still accumulate).  visible: DEVICE int32 [n] or NULL;
 * if given it is overwritten with 1 where some view's tiles_touched is
 * positive and 0 elsewhere -- the set the sparse Adam step of section 4.3
 * updates, as gs_mark_visible over the views would build it from zero. */
gs_status gs_project_bwd_views_store(int32_t n_views, const gs_view *views, const gs_raster_params *rp,
                                     const gs_gaussians *g, gs_gaussians *grads, void *ws, size_t ws_bytes,
                                     int32_t *visible, void *stream);

/* Rates and constants of the sparse Adam step of the joint optimisation
 * (section 4.3): one rate per parameter group -- means, log-scales,
 * quaternions, opacity logits, the degree-0 SH coefficients (planes 0..2 of
 * sh) and the higher-degree ones (planes 3..) -- Adam's beta1, beta2, eps
 * and step (>= 1), and the per-Gaussian rate decay that follows the step,
 * in (0, 1] (the joint-optimisation appendix). */
typedef struct {
  float lr_means, lr_log_scales, lr_quats, lr_opacity, lr_sh_dc, lr_sh_rest;
  float beta1, beta2, eps;
  int32_t step;
  float lr_decay;
} gs_adam_groups; /* HOST memory */

/* The store-form adjoint of the window followed by the sparse Adam step and
 * the rate decay, the step applied by the adjoint's last pass while each
 * Gaussian's gradients are still in registers (the gradients of the SH
 * coefficients never reach memory).  On return g, m1, m2 (the first and
 * second moments, same shapes as g), lr_scale and visible hold exactly what
 * gs_project_bwd_views_store (into grads, with visible), then
 * gs_adam_step on each group (visible, lr_scale, n_stride = n) and
 * gs_lr_decay (visible) would leave; each view's pose gradient is
 * accumulated as there.  grads is scratch (its contents on return are
 * unspecified); visible (DEVICE int32 [n]) is required and overwritten;
 * lr_scale (DEVICE float [n]) may be NULL (rate lr, no decay).  ws: the
 * gs_project_bwd_views_workspace(n, n_views) bytes.  g, m1, m2, lr_scale
 * are updated in place. */
gs_status gs_project_bwd_views_adam(int32_t n_views, const gs_view *views, const gs_raster_params *rp,
                                    gs_gaussians *g, gs_gaussians *m1, gs_gaussians *m2, float *lr_scale,
                                    const gs_adam_groups *opt, gs_gaussians *grads, void *ws, size_t ws_bytes,
                                    int32_t *visible, void *stream);

/* ---- loss, metrics and optimiser (helpers of the joint optimisation) ----
 * gs_loss_l1: over count values, sums[0] = sum |image - target|,
 * sums[1] = sum (image - target)^2 (double, DEVICE, overwritten), and if
 * dL_dimage is not NULL, dL_dimage = grad_scale * sign(image - target)
 * (sign(0) = 0).  ws: gs_loss_workspace(count) bytes. */
gs_status gs_loss_workspace(int64_t count, size_t *bytes);
gs_status gs_loss_l1(const float *image, const float *target, int64_t count, float grad_scale, float *dL_dimage,
                     double *sums, void *ws, size_t ws_bytes, void *stream);

/* gs_psnr: peak signal-to-noise ratio over count values (section 5
 * evaluates novel views by it; the joint optimisation logs it):
 * out[0] = 10 log10(peak^2 / MSE) in dB, +inf when the images are equal,
 * out[1] = MSE = sum (image - target)^2 / count, both summed in binary64
 * (DEVICE, double [2], overwritten).  count >= 1, peak > 0 (1 for [0, 1]
 * images).  ws: gs_psnr_workspace(count) bytes. */
gs_status gs_psnr_workspace(int64_t count, size_t *bytes);
gs_status gs_psnr(const float *image, const float *target, int64_t count, float peak, double *out, void *ws,
                  size_t ws_bytes, void *stream);

/* Number of NaN and infinite values among count floats (host out *n_bad);
 * synchronises the stream.  The counting behind GS_CHECK_FINITE, callable
 * on its own; shares the library's one device counter per GPU (calls are
 * serialised by a host lock). */
gs_status gs_count_nonfinite(const float *x, int64_t count, int64_t *n_bad, void *stream);

/* One Adam step (bias-corrected, step >= 1) on count floats:
 *   m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
 *   p -= lr_e (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 * Sparse form (section 4.3, sparse Adam): if visible is not NULL, element e
 * belongs to Gaussian e % n_stride and is left untouched (p, m, v) unless
 * visible[e % n_stride] != 0.  Per-Gaussian rates (section 4.3 and the
 * joint-optimisation appendix): if lr_scale [n_stride] is not NULL,
 * lr_e = lr * lr_scale[e % n_stride] (FP32 product), else lr_e = lr.
 * n_stride > 0 is required with either array.  In place; no workspace. */
gs_status gs_adam_step(float *param, const float *grad, float *m, float *v, int64_t count, float lr, float beta1,
                       float beta2, float eps, int32_t step, const int32_t *visible, const float *lr_scale,
                       int64_t n_stride, void *stream);

/* The per-Gaussian rate decay that follows a sparse step (the
 * joint-optimisation appendix): lr_scale[i] *= decay for every i with
 * visible[i] != 0 (every i if visible is NULL).  A Gaussian's factor starts
 * at 1 when it is introduced (the caller writes it), so after k steps that
 * processed it the factor is decay^k.  decay in (0, 1]. */
gs_status gs_lr_decay(float *lr_scale, const int32_t *visible, int64_t n, float decay, void *stream);

/* Pose from the continuous 6D rotation representation used for the camera
 * poses (section 4.3): x [V][9] = (a1, a2, t); R's columns are
 * b1 = a1/|a1|, b2 = unit(a2 - (b1.a2) b1), b3 = b1 x b2; pose [V][12] =
 * (R row-major, t).  gs_pose_6d_bwd maps dL/dpose [V][12] (double) to
 * dL/dx [V][9] (float, accumulated). */
gs_status gs_pose_from_6d(const float *x, float *pose, int32_t n_views, void *stream);
gs_status gs_pose_6d_bwd(const float *x, const double *dL_dpose, float *dL_dx, int32_t n_views, void *stream);

/* Zero `bytes` bytes of device memory with a kernel (no memset node, so the
 * call can sit inside a captured graph). */
gs_status gs_zero(void *ptr, size_t bytes, void *stream);

/* mask[i] |= (tiles_touched[i] > 0) over n Gaussians: the set a step
 * processed, which the sparse Adam step of section 4.3 updates. */
gs_status gs_mark_visible(const int32_t *tiles_touched, int64_t n, int32_t *mask, void *stream);

/* gs_filter3d_update: the 3D smoothing filter's sampling rates (section 4.3's
 * "proper filtering", Mip-Splatting): for each Gaussian, nu_max = max(nu_max,
 * fx / z) over the cameras whose image, widened by `guard` times its size
 * about its centre (1.15 in Mip-Splatting), holds the projected mean in front
 * of the near plane (binary64 on the binary32 means; nu_max [n] DEVICE,
 * in/out, 0 for a Gaussian no camera has seen); then, if filter3d is not
 * NULL, filter3d = (s_f / nu_max)^2, 0 where nu_max = 0 (s_f = 0.2 in
 * Mip-Splatting).  Call it with every new keyframe's camera.  cams: n_views
 * host structs (poses on the device).  Errors: GS_ERR_INVALID_ARG for NULL
 * arrays, guard < 1, s_f <= 0, a bad camera. */
gs_status gs_filter3d_update(const float *means, int64_t n, int32_t n_views, const gs_camera *cams, float guard,
                             float s_f, float *nu_max, float *filter3d, void *stream);

/* ---- multi-scale training (section 4.3) ------------------------------
 * Coarse-to-fine: a newly added image first trains at 2^l downsampling
 * (l = 3), one level less every five iterations until full size; the
 * target is the box-filtered image and the camera the matching coarse one.
 *
 * gs_downsample: out [C][H >> level][W >> level] with coarse pixel (x, y)
 * of plane c = mean (FP32 sum in row order, times 2^-2level) of in[c] over
 * rows 2^level y .. 2^level y + 2^level - 1 and the same columns of x; the
 * right and bottom remainders that do not fill a block are dropped.  in
 * [C][H][W], device memory; out must not overlap in.  level 0..4 (0 is a
 * copy).  Errors: GS_ERR_INVALID_ARG for bad sizes, NULL pointers, or an
 * image smaller than one block. */
gs_status gs_downsample(const float *in, int32_t channels, int32_t width, int32_t height, int32_t level, float *out,
                        void *stream);

/* The camera that renders the 2^level-downsampled image (host only, no GPU
 * work): width >> level, height >> level, f / 2^level, and
 * c' = (c + 1/2) / 2^level - 1/2 (pixel centres at integer coordinates: a
 * coarse pixel's centre is the centroid of its fine pixels' centres); the
 * pose pointer, near plane and background are copied.  out may equal cam. */
gs_status gs_camera_level(const gs_camera *cam, int32_t level, gs_camera *out);

/* Opacity culling (section 4.3, as in 3DGS): Gaussian i is kept iff
 * opacity_logits[i] >= thr, thr = binary32 rounding of ln(t / (1 - t))
 * computed in binary64 on the host, t = min_opacity in (0, 1) -- the test
 * sigmoid(logit) >= t taken on the logit in FP32.  keep_index [n] (device)
 * receives the kept indices in ascending order, *n_keep (host) their
 * number; entries past *n_keep are unspecified.  Reads the count back and
 * synchronises the stream once.  ws: gs_prune_workspace(n) bytes.
 * n <= 2^31 - 1. */
gs_status gs_prune_workspace(int64_t n, size_t *bytes);
gs_status gs_prune_opacity(const float *opacity_logits, int64_t n, float min_opacity, int32_t *keep_index,
                           int64_t *n_keep, void *ws, size_t ws_bytes, void *stream);

/* dst[p][j] = src[p][index[j]] for p < planes, j < m: src planes of stride
 * n_src, dst planes of stride m, device memory, not overlapping.  With
 * gs_prune_opacity's keep_index this compacts every parameter plane, Adam
 * moment and per-Gaussian rate to the kept Gaussians (planes <= 65535; an
 * index outside [0, n_src) gives 0). */
gs_status gs_gather_planes(const float *src, int64_t n_src, int32_t planes, const int32_t *index, int64_t m,
                           float *dst, void *stream);

/* ---- spawning (section 4.2) ---------------------------------------------
 * A new frame spawns primitives where its image has structure that the
 * current model does not render (Eq. 1-3):
 *   P_L(p) = min(|LoG * I|(p), 1), the L2 norm over R, G, B of the response
 *            of the input image I to a Laplacian-of-Gaussian filter;
 *   P~(p)  = the same quantity on the image rendered from the new view
 *            (absent on the first frame: P~ = 0);
 *   P_s(p) = max(P_L(p) - P~(p), 0), the spawn probability.
 * The filter: the analytic LoG of standard deviation sigma sampled on the
 * integer grid out to radius r = ceil(4 sigma), minus the taps' exactly
 * rounded mean (so they sum to zero), rounded to float32; replicated
 * borders.  The probability is computed in float32 in a fixed order (taps
 * row by row, each product rounded then added; squares of R, G, B added in
 * that order; correctly rounded sqrt), so every spawn decision below, an
 * integer function of it, is reproducible bit for bit.
 *
 * Selection (the paper samples pixels by P_s; the draws are fixed here):
 *   q(p) = floor(P_s(p) 2^24);
 *   GS_SPAWN_BERNOULLI: pixel p spawns iff u(p) < q(p), u(p) = the top 24
 *     bits of SplitMix64 (Steele, Lea, Flood 2014) of seed + p, p the flat
 *     pixel index v W + u;
 *   GS_SPAWN_FIXED_K: systematic sampling of K thresholds over the integer
 *     masses: S = sum q, o = top 24 bits of SplitMix64(seed),
 *     U = floor(S o / 2^24), t_j = floor((j S + U) / K), j = 0..K-1; a pixel
 *     spawns (once) if some t_j falls in [prefix(p), prefix(p) + q(p)).
 * Initialisation (the paper's direct rule): position at the pixel's depth D
 * on its ray, mean = R^T (D ((u - cx)/fx, (v - cy)/fy, 1) - t); isotropic
 * scale D / (2 f sqrt(max(P_L, min_prob))), f = sqrt(fx fy), the
 * nearest-neighbour distance of a Poisson process of intensity P_L per
 * pixel (Clark-Evans) in world units; rotation = the camera's axes (the
 * unit quaternion of R^T with w >= 0); opacity `opacity`; colour = the
 * pixel's, as the DC SH term (rgb - 0.5) 2 sqrt(pi), higher SH zero. */
typedef enum { GS_SPAWN_BERNOULLI = 0, GS_SPAWN_FIXED_K = 1 } gs_spawn_mode;

typedef struct {
  float sigma;      /* LoG standard deviation in pixels, (0, 2] (1) */
  int32_t mode;     /* gs_spawn_mode (GS_SPAWN_BERNOULLI) */
  int64_t k;        /* thresholds for GS_SPAWN_FIXED_K, >= 0 */
  uint64_t seed;    /* counter base of the draws (0) */
  float opacity;    /* initial opacity, (0, 1) (0.1) */
  float min_prob;   /* floor of P_L in the scale rule, > 0 (1e-4) */
} gs_spawn_params;  /* HOST memory */

void gs_default_spawn_params(gs_spawn_params *sp);

/* The float32 LoG taps: writes (2r+1)^2 row-major values into HOST taps
 * (room for 289) and r into HOST *radius.  Host only, no device work. */
gs_status gs_spawn_log_taps(float sigma, float *taps, int32_t *radius);

/* image, rendered: [3][H][W] float32 in [0, 1] (rendered may be NULL: first
 * frame).  Writes p_s [H][W] and, if not NULL, p_l [H][W]. */
gs_status gs_spawn_probability(const gs_camera *cam, const float *image, const float *rendered,
                               const gs_spawn_params *sp, float *p_l, float *p_s, void *stream);

/* Selects pixels from p_s [H][W] and writes their flat indices in
 * increasing order to pixels [capacity], the count to HOST *n_selected.
 * Synchronises the stream once (to read the count).  If the count exceeds
 * capacity: GS_ERR_CAPACITY, *n_selected = the count, pixels unwritten.
 * ws: gs_spawn_select_workspace(W, H) bytes. */
gs_status gs_spawn_select_workspace(int32_t width, int32_t height, size_t *bytes);
gs_status gs_spawn_select(const gs_camera *cam, const float *p_s, const gs_spawn_params *sp, int64_t capacity,
                          int32_t *pixels, int64_t *n_selected, void *ws, size_t ws_bytes, void *stream);

/* Writes the rule's parameters of `count` primitives spawned at pixels
 * [count] into entries [offset, offset + count) of out (planes of stride
 * out->n; offset + count > out->n is GS_ERR_CAPACITY).  image [3][H][W],
 * depth [H][W] (> 0 at the selected pixels), p_l [H][W]. */
gs_status gs_spawn_rule(const gs_camera *cam, const float *image, const float *depth, const float *p_l,
                        const int32_t *pixels, int64_t count, const gs_spawn_params *sp, gs_gaussians *out,
                        int64_t offset, void *stream);

/* ---- learned spawn initialisation ----------------------------------------
 * A 196 -> 64 -> 64 -> 7 MLP with exact GELU, 0.5 x (1 + erf(x / sqrt 2)),
 * predicts residuals over the rule above for a primitive spawned at pixel
 * p = (u, v): outputs 0..2 are added to the three log-scales (camera x, y,
 * ray axis), 3 to the opacity logit, 4..6 to the colour (so the DC SH term
 * moves by 2 sqrt(pi) times them).  Inputs: the 7x7 RGB patch centred on p
 * (row-major, channel-last: input (3 (7 dy + dx) + c)), then the 7x7 depth
 * patch as log(D(q) / D(p)) (input 147 + 7 dy + dx); replicated borders.
 * Parameters theta [GS_MLP_PARAMS] float32: W1 [64][196], b1 [64],
 * W2 [64][64], b2 [64], W3 [7][64], b3 [7] (row-major: layer = W x + b).
 * Inference runs on BF16 matrix cores (inputs, weights and hidden
 * activations rounded to bfloat16 to nearest-even, FP32 accumulation);
 * training in FP32. */
#define GS_MLP_INPUTS 196
#define GS_MLP_OUTPUTS 7
#define GS_MLP_PARAMS 17223

/* Bytes of the packed BF16 inference weights. */
size_t gs_mlp_packed_bytes(void);
/* theta [GS_MLP_PARAMS] -> packed [gs_mlp_packed_bytes()] (device). */
gs_status gs_mlp_pack_bf16(const float *theta, void *packed, void *stream);
/* features [count][196] of the pixels [count] (flat indices) of a frame:
 * image [3][H][W], depth [H][W] > 0. */
gs_status gs_mlp_features(const gs_camera *cam, const float *image, const float *depth, const int32_t *pixels,
                          int64_t count, float *features, void *stream);
/* out [count][7] = MLP(features [count][196]) on the BF16 path. */
gs_status gs_mlp_forward_bf16(const void *packed, const float *features, int64_t count, float *out, void *stream);
/* Adds the MLP's residuals, computed from the frame at pixels [count], onto
 * the parameters of entries [offset, offset + count) of out, which hold the
 * rule's values (gs_spawn_rule).  Features are gathered inside the kernel. */
gs_status gs_spawn_mlp(const gs_camera *cam, const float *image, const float *depth, const int32_t *pixels,
                       int64_t count, const void *packed, gs_gaussians *out, int64_t offset, void *stream);

/* One FP32 training step on a batch: loss = mean over batch x 7 of
 * (MLP(features) - targets)^2 (targets [batch][7]); its gradient is written
 * to grad [GS_MLP_PARAMS] if not NULL and the loss (before the update) to
 * *loss (device float) if not NULL; then, if lr != 0, one Adam step on
 * theta with moments m, v (the update of gs_adam_step, step >= 1).
 * ws: gs_mlp_train_workspace(batch) bytes.  batch 1 .. 2^24. */
gs_status gs_mlp_train_workspace(int64_t batch, size_t *bytes);
gs_status gs_mlp_train_step(float *theta, float *m, float *v, const float *features, const float *targets,
                            int64_t batch, float lr, float beta1, float beta2, float eps, int32_t step, float *loss,
                            float *grad, void *ws, size_t ws_bytes, void *stream);

/* The whole spawn step of a new frame: probability, selection, the rule and,
 * if mlp_packed is not NULL, the learned residuals.  Spawned primitives are
 * written to out entries [offset, offset + *n_spawned); the selection may
 * hold at most out->n - offset of them (else GS_ERR_CAPACITY with
 * *n_spawned = the count, out untouched).  rendered may be NULL (first
 * frame).  Synchronises the stream once.
 * ws: gs_spawn_init_workspace(W, H, out->n - offset) bytes. */
gs_status gs_spawn_init_workspace(int32_t width, int32_t height, int64_t capacity, size_t *bytes);
gs_status gs_spawn_init(const gs_camera *cam, const float *image, const float *depth, const float *rendered,
                        const gs_spawn_params *sp, const void *mlp_packed, gs_gaussians *out, int64_t offset,
                        int64_t *n_spawned, void *ws, size_t ws_bytes, void *stream);

/* ---- guided-matching depth (the appendix on depth for new primitives) ----
 * Depth for the primitives a frame spawns (section 4.2), found around the
 * monocular depth Z*.  Per pixel (x, y) of frame i:
 *   candidates d_k = lo + k (hi - lo) / (n_cand - 1), lo = max(1/Z* - r_inv,
 *   1e-3), hi = 1/Z* + r_inv (inverse depths; the paper's r_inv = 0.1);
 *   the neighbour j (of n_nb) whose reprojections of d_0 and d_{n-1} lie
 *   farthest apart in pixels with both inside [0, W-1] x [0, H-1] and in
 *   front of camera j (ties: the lower j; none: no estimate);
 *   reprojection p = R_j (K^-1 (x, y, 1) / d_k) + t_j, (u, v) = (fx p_x /
 *   p_z + cx, fy p_y / p_z + cy), shared intrinsics;
 *   C_k = <F_i(x, y), F_j(u, v)>, F_j bilinear with pixel centres at
 *   integers and taps outside the image counted as 0; a candidate behind
 *   camera j has none;
 *   k* = argmax C_k (lowest k on ties), delta = (C_{k*-1} - C_{k*+1}) /
 *   (2 (C_{k*-1} - 2 C_{k*} + C_{k*+1})) when both neighbours exist and the
 *   denominator is negative, else 0; depth = 1 / (lo + (k* + delta)(hi -
 *   lo) / (n_cand - 1)).
 * feat_i: FP16 [H][W][channels] (channel-last, 16-byte aligned), channels
 * in {8, 16, 32, 64}; feat_nb: HOST array of n_nb (1..4) DEVICE pointers of
 * the same layout; rel_poses: HOST [n_nb][12] = R (row-major) then t of
 * each neighbour's camera relative to frame i's; zmono [H][W] FP32.
 * Outputs [H][W]: depth (NaN: no estimate, also where Z* is not positive
 * and finite), best = k* (optional, -1: none), choice = j (optional, -1).
 * Inner products in FP32 from exact FP16 products.  n_cand 3..1024. */
gs_status gs_guided_depth(int32_t width, int32_t height, int32_t channels, float fx, float fy, float cx, float cy,
                          const void *feat_i, int32_t n_nb, const void *const *feat_nb, const float *rel_poses,
                          const float *zmono, int32_t n_cand, float r_inv, float *depth, int32_t *best,
                          int32_t *choice, void *stream);

/* ---- anchors (section 4.4) ------------------------------------------------
 * gs_anchor_sizes: the creation trigger's per-Gaussian test.  A primitive's
 * size from a camera is S / D, S its scale and D the distance of its mean to
 * the camera centre C = -R^T t (pose: HOST [12], R row-major then t, the
 * world -> camera pose of the previous camera); S is read as the largest of
 * the three axis scales, and the test is f S < tau D in FP64 with f the
 * focal length in pixels and tau the threshold in pixels (the paper's
 * tau_min = 1).  flags [n] (optional) receives 1 / 0; count (DEVICE, one
 * uint64) receives the number of small Gaussians (overwritten, not
 * accumulated).  An anchor is created when count > 0.4 n.
 * gs_anchor_blend_weight (host only): the nearer anchor's weight for two
 * anchors at distances d1 <= d2 with overlap o in (0, 0.5): 1 for
 * r = d1 / d2 < 1 - o, else 1 - (r - (1 - o)) 0.5 / o (the other anchor
 * takes 1 - w).
 * gs_scale_opacity: out[i] = logit(w sigmoid(logits[i])) in FP64, w in
 * [0, 1] (w = 0 gives -inf: the Gaussian is culled); out may equal logits. */
gs_status gs_anchor_sizes(const float *means, const float *log_scales, int64_t n, const float *pose, float f,
                          float tau, int32_t *flags, unsigned long long *count, void *stream);
gs_status gs_anchor_blend_weight(float d1, float d2, float overlap, float *w);
gs_status gs_scale_opacity(const float *logits, int64_t n, float w, float *out, void *stream);

/* ---- anchor merging (section 4.4, "Clustering and Primitive Merging") ---
 * When an anchor is created, a random share 1/(k+1) of the primitives that
 * look too fine (fine[i] != 0, e.g. the flags of gs_anchor_sizes) is
 * selected and each selected primitive is merged with its k nearest
 * neighbours among the other too-fine primitives (k = 3 in the paper); all
 * other primitives are kept, in their order, as the new active set.
 *
 * gs_anchor_merge_plan (synchronises the stream twice for counts):
 *   selection  cls[i] = 1 (selected) iff fine[i] and the top 24 bits of
 *              SplitMix64(seed + i) < floor(2^24 / (k+1)); 2 for the other
 *              fine primitives (candidates); 0 otherwise.
 *   nbr [n][k] for a selected i its k nearest candidates by the binary64
 *              squared distance (dx dx + dy dy) + dz dz of the binary32
 *              means, ascending, ties to the lower index (exactly the
 *              brute-force result), -1 where fewer exist; -1 rows elsewhere.
 *   owner [n]  for a candidate, the selected primitive it joins -- of those
 *              that list it, the one with the smallest (binary32 d2, index)
 *              -- else -1.
 *   new_index [n]  position in the new active set, -1 for an absorbed
 *              candidate; keep_index [n]: the first *n_keep entries are the
 *              ascending indices of the kept primitives.
 *   k in [1, 8]; ws: gs_anchor_merge_workspace(n) bytes.  Errors:
 *   GS_ERR_INVALID_ARG for NULL arrays (n > 0), k out of range, n >= 2^31
 *   or a candidate mean that is not finite.
 * gs_anchor_merge_apply: writes the new active set into out (out->n =
 *   *n_keep, same SH degree): the kept primitives gathered, and every
 *   selected primitive that received a neighbour replaced by the merge of
 *   its group (FP64): weights w = opacity * s_x s_y s_z, the weighted mean,
 *   the weighted second moment about it (member covariances plus spreads) as
 *   the covariance (its eigenvectors -> rotation, half log-eigenvalues ->
 *   log-scales), SH coefficients averaged with the same weights, opacity
 *   min(0.99, W / sqrt(det Sigma)).  merged [out->n] (optional) is set to 1
 *   at the merged entries, 0 elsewhere, so the caller can reset their
 *   optimiser state (gs_gather_planes with keep_index carries the rest). */
gs_status gs_anchor_merge_workspace(int64_t n, size_t *bytes);
gs_status gs_anchor_merge_plan(const gs_gaussians *g, const int32_t *fine, int32_t k, uint64_t seed, int32_t *cls,
                               int32_t *nbr, int32_t *owner, int32_t *new_index, int32_t *keep_index,
                               int64_t *n_keep, void *ws, size_t ws_bytes, void *stream);
gs_status gs_anchor_merge_apply(const gs_gaussians *g, const int32_t *cls, const int32_t *nbr, const int32_t *owner,
                                const int32_t *new_index, const int32_t *keep_index, int32_t k, gs_gaussians *out,
                                int32_t *merged, void *stream);

/* planes [n_planes][n]: planes[p][i] = value wherever mask[i] != 0 (e.g. the
 * Adam moments of the merged entries of gs_anchor_merge_apply, reset to 0). */
gs_status gs_masked_fill(float *planes, int64_t n, int32_t n_planes, const int32_t *mask, float value,
                         void *stream);

/* ---- anchor storage (section 4.4) ----------------------------------------
 * An anchor stores the active Gaussians, their optimisation state and the
 * keyframes they were optimised with in CPU RAM, off the GPU.
 * gs_anchor_offload copies n_planes DEVICE arrays (src[p], bytes[p] bytes)
 * into one HOST block, each at a 256-byte aligned offset
 * (gs_anchor_host_bytes gives the block size); gs_anchor_reload copies them
 * back into dst[p].  Both are asynchronous on `stream` (a side stream keeps
 * them beside the optimisation); for the copies to be asynchronous the host
 * block must be pinned (page-locked) memory the caller allocated.  The host
 * block must not be read or freed before the stream has passed the call. */
size_t gs_anchor_host_bytes(int32_t n_planes, const size_t *bytes);
gs_status gs_anchor_offload(int32_t n_planes, const void *const *src, const size_t *bytes, void *host, void *stream);
gs_status gs_anchor_reload(int32_t n_planes, void *const *dst, const size_t *bytes, const void *host, void *stream);

/* ---- spatial cells of a large scene (section 4.4) --------------------------
 * The scalable construction keeps on the device only what the current views
 * need and parks the rest in CPU RAM.  For a scene too large to stay
 * resident the Gaussians are grouped into spatial cells by Lloyd's k-means
 * over their means; a cell is copied to the device when its bounding sphere
 * meets a view's frustum.
 *
 * gs_cells_assign: labels[i] = the nearest of the k centroids (DEVICE
 *   double [k][3]) to mean i, by (dx dx + dy dy) + dz dz in binary64 on the
 *   binary32 means with every operation rounded on its own; ties go to the
 *   lower centroid.  means [3][n] DEVICE; 1 <= k <= 1024.
 * gs_cells_kmeans: `iters` Lloyd iterations (assign, then move each
 *   centroid to the binary64 mean of its members; a centroid without
 *   members stays), then a final assignment.  init != 0 starts from the
 *   means at indices floor((j + 1/2) n / k), else from the caller's
 *   centroids.  Outputs (DEVICE): centroids [k][3] (in/out), labels [n];
 *   if not NULL, order [n] = the indices stably sorted by label and
 *   offsets [k + 1] = each cell's first position in that order
 *   (offsets[k] = n).  The sums are taken in a fixed order (per 4096-mean
 *   chunk in index order, then over the chunks in order): the result does
 *   not depend on scheduling.  1 <= k <= min(n, 1024), n < 2^31.
 *   ws: gs_cells_kmeans_workspace(n, k) bytes.
 * gs_cells_spheres: radius[j] = max over cell j's members of the distance
 *   from centroid j to the mean, plus margin times the largest exp(log
 *   scale) of its members (0 for an empty cell).  log_scales [3][n].
 *   ws: gs_cells_spheres_workspace(n, k) bytes.
 * gs_cells_visible: visible[j] = 1 iff sphere j (centre centroids[j],
 *   radius[j]) reaches in front of the camera's near plane and meets the
 *   four side planes of its image frustum widened by `guard` half-FOVs
 *   (the projection's guard band), in binary64; else 0.
 * Errors: GS_ERR_INVALID_ARG for NULL arrays, sizes out of range, a bad
 * camera; GS_ERR_WORKSPACE for a short workspace. */
gs_status gs_cells_assign(const float *means, int64_t n, const double *centroids, int32_t k, int32_t *labels,
                          void *stream);
gs_status gs_cells_kmeans_workspace(int64_t n, int32_t k, size_t *bytes);
gs_status gs_cells_kmeans(const float *means, int64_t n, int32_t k, int32_t iters, int32_t init, double *centroids,
                          int32_t *labels, int32_t *order, int64_t *offsets, void *ws, size_t ws_bytes,
                          void *stream);
gs_status gs_cells_spheres_workspace(int64_t n, int32_t k, size_t *bytes);
gs_status gs_cells_spheres(const float *means, const float *log_scales, int64_t n, const int32_t *labels,
                           const double *centroids, int32_t k, float margin, double *radius, void *ws,
                           size_t ws_bytes, void *stream);
gs_status gs_cells_visible(const double *centroids, const double *radius, int32_t k, const gs_camera *cam,
                           float guard, int32_t *visible, void *stream);

/* Residency of cells (the device holds the cells the current views need,
 * the CPU RAM all of them).  gs_copy_rows: `height` rows of `width` bytes,
 * row r from src + r spitch to dst + r dpitch, asynchronously on the stream
 * (either side may be pinned host memory or device memory; a cell's
 * parameter and optimiser rows move in one call).  gs_fill_f32: count floats
 * of DEVICE memory set to value (e.g. an opacity logit that culls the
 * unused columns of a page).  Errors: GS_ERR_INVALID_ARG for NULL pointers
 * or a row wider than its pitch; GS_ERR_HIP if the copy fails. */
gs_status gs_copy_rows(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                       void *stream);
gs_status gs_fill_f32(float *dst, int64_t count, float value, void *stream);

/* ---- mini bundle adjustment (section 4.1, appendix "Initial Pose
 * Estimation") ------------------------------------------------------------
 * Levenberg-Marquardt as the appendix states it: damping lambda from 1e-5,
 * divided by 2 after a step that lowers the cost (the step is kept),
 * multiplied by 2 otherwise (the step is dropped); damped normal equations
 * (J^T W J + lambda diag(J^T W J)) delta = -J^T W r (a variable none of whose
 * observations is kept holds still).  Robustness: the Huber loss of each
 * observation's reprojection error e (threshold huber_delta pixels) and the
 * rejection of the observations with e > median + 4 MAD of the errors at
 * the iterate.  Poses are world->camera [R | t] (row-major R, then t) in
 * FP64, updated by left perturbations exp(xi^) T; the pinhole model is the
 * rasterizer's.  Each call is a fixed-size problem that runs whole on the
 * device (one launch per stage, all iterations inside).
 *
 * gs_pose_ransac: the pose of a new frame from K 3D-2D correspondences
 *   (X [3][K] world points, uv [2][K] pixels, DEVICE float32; K <= 8192):
 *   n_hyp hypotheses, each from the previous pose pose0 (HOST double[12])
 *   run hyp_iters plain LM iterations on `sample` correspondences drawn by
 *   the counter-based SplitMix64 stream (draw c of hypothesis h:
 *   splitmix64(seed + h 2^32 + c) mod K, repeats skipped) and count the
 *   correspondences in front of the camera with error < tau; the hypothesis
 *   with most inliers (the first on ties) is refined by refine_iters robust
 *   LM iterations on its inliers.  Out (DEVICE): inliers [K] (1 / 0 at the
 *   winner, before refinement), n_inliers [1], pose_out double[12],
 *   pose_out32 float[12], hyp_count [n_hyp] (optional).  ws:
 *   gs_pose_ransac_workspace(n_hyp) bytes.
 * gs_ba_bootstrap: focal length (fx = fy, principal point at the image
 *   centre), the poses of views 1..V-1 (view 0 is the identity) and P points
 *   seen in every view, from f = 0.7 width, identity poses and points at depth
 *   1 along view 0's rays: uv [V][2][P] DEVICE float32 (2 <= V <= 8, V P <=
 *   8192).  The points are eliminated per point (3 x 3 blocks) and the
 *   reduced camera system is solved by Cholesky.  The rejection applies from
 *   iteration mad_from on (< 0: iters / 2; the Huber loss throughout).  Out
 *   (DEVICE, FP64): f_out [1], pose_out [V][12], X_out [3][P], trace
 *   [iters][3] (cost, candidate cost, lambda per iteration; optional).  ws:
 *   gs_ba_bootstrap_workspace(V, P) bytes. */
gs_status gs_pose_ransac_workspace(int32_t n_hyp, size_t *bytes);
gs_status gs_pose_ransac(const float *X, const float *uv, int64_t K, float fx, float fy, float cx, float cy,
                         const double *pose0, int32_t n_hyp, int32_t sample, int32_t hyp_iters, float tau,
                         int32_t refine_iters, float huber_delta, uint64_t seed, int32_t *inliers, int32_t *n_inliers,
                         double *pose_out, float *pose_out32, int32_t *hyp_count, void *ws, size_t ws_bytes,
                         void *stream);
gs_status gs_ba_bootstrap_workspace(int32_t n_views, int32_t n_points, size_t *bytes);
gs_status gs_ba_bootstrap(const float *uv, int32_t n_views, int32_t n_points, int32_t width, int32_t height,
                          int32_t iters, int32_t mad_from, float huber_delta, double *f_out, double *pose_out,
                          double *X_out, double *trace, void *ws, size_t ws_bytes, void *stream);

/* ---- measurement probes --------------------------------------------------
 * The achievable rates on the device, reported beside the datasheet peaks
 * that the roofline fractions use.
 * gs_probe_copy: dst = src over `bytes` bytes with 16-byte loads and
 * stores (2 x bytes of HBM traffic); bytes and both pointers 16-byte
 * multiples, device memory, not overlapping.
 * gs_probe_valu: blocks x 256 lanes each run iters x 8 independent chains of
 * one VALU operation -- kind 0: v_fma_f32 (one lane-op per FMA), kind 1:
 * v_exp_f32 -- and write one float per lane to out [blocks * 256]. */
gs_status gs_probe_copy(const void *src, void *dst, size_t bytes, void *stream);
gs_status gs_probe_valu(int32_t kind, int32_t blocks, int32_t iters, float *out, void *stream);

/* ---- profiling ----------------------------------------------------------
 * When enabled, every kernel launch is bracketed with HIP events on its
 * stream; gs_profile_read sums the elapsed milliseconds of all launches of
 * the named kernel since the last reset (synchronising on its events).
 * Not thread-safe. */
void gs_profile_enable(int on);
/* Restricts the bracketing to the kernels named in a comma-separated list
 * (HOST string; NULL or "" = every kernel), so that a timed run pays for
 * the events of the kernels it reports only. */
void gs_profile_select(const char *names);
void gs_profile_reset(void);
gs_status gs_profile_read(const char *kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* GS_API_H */
