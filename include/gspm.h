/*
 * gspm.h -- C ABI of the MI355X (gfx950) differentiable Gaussian pointmap rasterizer.
 *
 * The library renders a set of 3D Gaussians into V views (keyframes) and returns, per
 * view, the composited colour (Sec. 3.1, Eq. 2), depth (Sec. 3.2.1, Eq. 3), alpha and
 * the "3D Gaussian pointmap" (the alpha-composited Gaussian centres, in the world or
 * camera frame, or the depth back-projection of Sec. 3.2.1, Eq. 4-5).  Its backward
 * pass returns gradients with respect to the Gaussian parameters (position, rotation,
 * scale, opacity and colour, Sec. 3.1) and to each view's SE(3) pose through the
 * projected means and covariances (Sec. 3.2.2, Eq. 11).  A per-patch least-squares
 * scale aligns a prior pointmap to the rendered one (Sec. 3.3.1), and the mapping loss
 * of Eq. 17 (photometric Eq. 10 + pointmap Eq. 15 terms) has a fused gradient kernel.
 *
 * Conventions shared by every call:
 *   - All arrays are float32 device memory unless marked "host".  Gaussian parameters
 *     are planar structure-of-arrays: means[3][n], log_scales[3][n], quats[4][n]
 *     (w, x, y, z, any norm), opacity_logit[n], rgb[3][n] (degree-0 colour, no
 *     activation).  Activated values: scale = exp(log_scale), rotation = the unit
 *     quaternion's matrix, opacity = sigmoid(logit).
 *   - Poses T_cw are device [V][12], row-major 3x4 [R | t] mapping world to camera
 *     (x right, y down, z forward).  Keeping them on the device lets a captured HIP
 *     graph see pose updates made in place.
 *   - Intrinsics are host structs.  Pixel (i, j) (i = column, j = row) is sampled at
 *     exactly (i, j), as Eq. 4 writes it.
 *   - Images of the V views are packed back to back in view order; view v starts at
 *     pixel offset P_v = sum_{u < v} W_u H_u, so its planar channel c of a 3-channel
 *     image sits at element 3 P_v + c H_v W_v + j W_v + i, and a 1-channel image at
 *     P_v + j W_v + i.
 *   - Every call is asynchronous on the given stream (a hipStream_t passed as void*;
 *     NULL is the null stream).  Argument errors are detected on the host before any
 *     launch and returned immediately; nothing is launched then.
 *   - Ownership: the caller owns every input, output, gradient and frame-state buffer.
 *     A context owns only scratch memory (sort buffers, per-record gradients, partial
 *     sums); it grows that scratch with hipMalloc when a call needs more, so calls that
 *     must not allocate (graph capture) should follow gspm_reserve with large enough
 *     capacities.
 *   - Gradient outputs are accumulated (+=), so one Gaussian set can be shared across
 *     calls; the caller zeroes them (or sets settings.grads_overwrite, which makes the
 *     backward write them instead).
 *   - A context is not thread safe and its calls must be ordered on one stream.
 */
#ifndef GSPM_H
#define GSPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define GSPM_API __attribute__((visibility("default")))
#else
#define GSPM_API
#endif

typedef enum {
    GSPM_OK = 0,
    GSPM_ERR_INVALID_ARG = 1, /* a pointer, size or setting is out of range */
    GSPM_ERR_CAPACITY = 2,    /* the tile-pair list did not fit the frame state */
    GSPM_ERR_HIP = 3,         /* a HIP runtime call failed (message in gspm_last_error) */
    GSPM_ERR_INTERNAL = 4
} gspm_status;

#define GSPM_MAX_VIEWS 32

typedef struct gspm_ctx gspm_ctx;

/* Gaussian set (device, planar SoA as described above). */
typedef struct {
    const float *means;
    const float *log_scales;
    const float *quats;
    const float *opacity_logit;
    const float *rgb;
    int64_t n;
} gspm_gaussians;

/* Pinhole intrinsics of one view (host): K = [[fx, 0, cx], [0, fy, cy], [0, 0, 1]] (Eq. 4). */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
} gspm_intrinsics;

/* The window of views rendered by one call. */
typedef struct {
    int32_t n_views;              /* 1 .. GSPM_MAX_VIEWS */
    const gspm_intrinsics *intr;  /* host [n_views] */
    const float *T_cw;            /* device [n_views][12] */
} gspm_views;

/* Rasterizer settings.  The paper fixes none of these numerically; each one is the
 * caller's choice.  Defaults used by the Python layer are given in brackets. */
typedef struct {
    int32_t tile;            /* tile edge in pixels: 8, 16 or 32 [16] */
    int32_t sort_digit_bits; /* largest radix-sort digit width, 4..8 [8]; each sort uses the
                                fewest passes this allows, with the bits spread evenly */
    int32_t pointmap_frame;  /* 0 world-frame composited centres, 1 camera frame,
                                2 depth back-projection D K^-1 [i, j, 1]^T (Eq. 5) [1] */
    int32_t pixels_per_lane; /* pixels each lane of the raster kernels owns; supported
                                (tile, pixels_per_lane): (8,1) (16,1) (16,2) (16,4) (32,1)
                                (32,2) (32,4) [1] */
    float near_z;            /* Gaussians with camera depth <= near_z are dropped [0.2] */
    float alpha_min;         /* fragments with alpha < alpha_min are skipped [1/255] */
    float alpha_max;         /* alpha is clamped to alpha_max [0.99] */
    float t_min;             /* compositing stops before transmittance drops below t_min [1e-4] */
    float eps2d;             /* low-pass added to the 2D covariance, px^2 [0.3] */
    float jac_clamp;         /* x/z, y/z clamped to jac_clamp * half FOV in the Jacobian [1.3] */
    float bg[3];             /* background colour added as T_final * bg [0] */
    int32_t mark_visible;    /* nonzero: the forward records which (Gaussian, view) records
                                contribute to at least one pixel, for gspm_covisibility [0] */
    int32_t count_work;      /* nonzero: the forward also counts each pixel's contributing
                                fragments, which gspm_frame_work reports [0] */
    int32_t bwd_lane_reduce; /* at one pixel per lane, the backward sums each record's
                                values over a wave's pixels with the matrix cores (0) or
                                with a cross-lane reduce-scatter (nonzero), the form it
                                always uses at 2 and 4 pixels per lane; the results agree
                                to float rounding [0] */
    int32_t grads_overwrite; /* nonzero: gspm_render_backward and gspm_pose_backward write the
                                parameter and pose gradients (0 where none flows) instead of
                                adding them to the arrays' contents, so a training loop
                                need not clear them first [0] */
} gspm_settings;

/* Per-view packed output planes (device): rgb [3][H][W], depth [H][W] (Eq. 3, not
 * normalised by alpha), alpha [H][W] = 1 - T_final, pointmap [3][H][W]. */
typedef struct {
    float *rgb;
    float *depth;
    float *alpha;
    float *pointmap;
} gspm_images;

/* Same planes, read-only (forward outputs and upstream gradients of the backward). */
typedef struct {
    const float *rgb;
    const float *depth;
    const float *alpha;
    const float *pointmap;
} gspm_const_images;

/* Gradient outputs (device, accumulated), same shapes as gspm_gaussians.  Any pointer
 * may be NULL to skip that parameter. */
typedef struct {
    float *means;
    float *log_scales;
    float *quats;
    float *opacity_logit;
    float *rgb;
} gspm_gaussian_grads;

/* ---- context ----------------------------------------------------------------------- */

GSPM_API gspm_status gspm_create(gspm_ctx **out);
GSPM_API void gspm_destroy(gspm_ctx *ctx);

/* Grow the context's scratch so that later calls with at most max_records
 * Gaussian-view records (n * n_views), max_pairs tile pairs and max_tiles tiles
 * allocate nothing.  Sizes never shrink.  Both counts must be below 2^30 (the radix
 * sorts' limit; GSPM_ERR_INVALID_ARG otherwise). */
GSPM_API gspm_status gspm_reserve(gspm_ctx *ctx, int64_t max_records, int64_t max_pairs, int64_t max_tiles);

/* Bytes of the caller-owned frame state that carries everything the backward needs
 * from its forward (projected records, sorted tile pairs, tile ranges, per-pixel
 * transmittance and last fragment, and per wave of a tile one bit per tile pair that
 * marks the pairs its pixels accepted).  max_pairs bounds the tile-pair list. */
GSPM_API int64_t gspm_frame_state_bytes(const gspm_views *views, int64_t n_gaussians, int64_t max_pairs,
                               int32_t tile);

/* ---- rendering (Sec. 3.1 Eq. 1-2, Sec. 3.2.1 Eq. 3-5) ------------------------------- */

/* Render all views.  frame_state: device buffer of frame_state_bytes >=
 * gspm_frame_state_bytes(views, g->n, max_pairs, s->tile), written by this call.
 * g->n * views->n_views must be below 2^30, and the pair capacity taken from the
 * buffer's size is capped at 2^30 - 1 (the radix sorts' limit).
 * If the views need more than max_pairs tile pairs the images are incomplete and the
 * frame state records the overflow: gspm_frame_status then returns GSPM_ERR_CAPACITY
 * with the number of pairs needed. */
GSPM_API gspm_status gspm_render_forward(gspm_ctx *ctx, const gspm_gaussians *g, const gspm_views *views,
                                const gspm_settings *s, const gspm_images *out, void *frame_state,
                                int64_t frame_state_bytes, void *stream);

/* Synchronise the stream and read the frame state's header: *pairs = tile pairs the
 * forward produced (or needed).  Returns GSPM_ERR_CAPACITY on overflow, and
 * GSPM_ERR_INVALID_ARG if a backward refused the frame state (see gspm_render_backward). */
GSPM_API gspm_status gspm_frame_status(const void *frame_state, void *stream, int64_t *pairs);

/* Synchronise the stream and report the work of a forward in out[5]: out[0] = tile pairs,
 * out[1] = contributing fragments (Gaussian-pixel pairs composited with alpha >=
 * alpha_min before the transmittance floor), out[2] = sum over pixels of the list
 * entries up to each pixel's last contributing fragment, out[3] = (wave, list entry)
 * pairs the forward's waves walked (those that passed the wave's rectangle test; each
 * evaluates 64 lanes), out[4] = the walked pairs that a live pixel of the wave accepted
 * (those the backward walks).  The frame state must come from a forward with the same
 * views, n_gaussians and tile, run with settings.count_work != 0 (GSPM_ERR_INVALID_ARG
 * otherwise). */
GSPM_API gspm_status gspm_frame_work(gspm_ctx *ctx, const gspm_views *views, int64_t n_gaussians, int32_t tile,
                                     const void *frame_state, void *stream, int64_t *out);

/* ---- gradients (Sec. 3.1 parameters; Sec. 3.2.2 Eq. 11 pose) ------------------------ */

/* Backward of gspm_render_forward for upstream gradients grad_out (same planes as the
 * outputs; any plane may be NULL for zero).  fwd_out are the forward's outputs (rgb,
 * depth, alpha and pointmap are read).  grads: accumulated parameter gradients (written
 * instead, 0 where none flows, with settings.grads_overwrite).
 * pose_grad: device [V][6] accumulated (or written), or NULL; it is d L / d xi at xi = 0 for the
 * left perturbation T_cw <- Exp(xi) T_cw, xi = (rho, phi) with the translation first.
 *
 * Same-settings contract: g, views (sizes, intrinsics and the poses in T_cw) and the
 * settings must be those of the forward that wrote frame_state; only pixels_per_lane and
 * bwd_lane_reduce may differ.  The views' sizes, the Gaussian count, the tile and the
 * pointmap frame are checked on the device against the frame state's header (so the
 * check also holds inside a captured graph), together with the forward's overflow and
 * sort-stall flags: on a mismatch, or on an incomplete forward, the backward reads
 * nothing of the frame state, adds nothing to grads and pose_grad (writes zeros with
 * settings.grads_overwrite), and marks the frame
 * state so that gspm_frame_status returns GSPM_ERR_INVALID_ARG until the next forward
 * into it.  Changed poses or parameters are not detected: the gradients are then those
 * of a render that was not made. */
GSPM_API gspm_status gspm_render_backward(gspm_ctx *ctx, const gspm_gaussians *g, const gspm_views *views,
                                 const gspm_settings *s, const gspm_const_images *fwd_out,
                                 const gspm_const_images *grad_out, const void *frame_state,
                                 const gspm_gaussian_grads *grads, float *pose_grad, void *stream);

/* Pose-only backward (Gaussians frozen, the tracking loop of Sec. 3.2.2): writes
 * pose_grad [V][6] (accumulated, or written with settings.grads_overwrite) and skips the
 * colour and opacity terms. */
GSPM_API gspm_status gspm_pose_backward(gspm_ctx *ctx, const gspm_gaussians *g, const gspm_views *views,
                               const gspm_settings *s, const gspm_const_images *fwd_out,
                               const gspm_const_images *grad_out, const void *frame_state,
                               float *pose_grad, void *stream);

/* ---- patch scale and mapping loss (Sec. 3.3.1, Eq. 10, 15, 17) --------------------- */

/* Per-patch least-squares scale aligning a prior pointmap Xp to the rendered one Xr:
 * patch in [1, 64]; for every patch x patch block of every view (partial at the right/bottom border),
 * scale = sum(Xr . Xp) / sum(|Xp|^2) over pixels with mask != 0 (mask NULL = all), or
 * 1 when sum(|Xp|^2) = 0.  Xr, Xp: packed [3][H][W] per view; mask: packed [H][W] or
 * NULL.  scale_out (float) and count_out (int32, may be NULL): per view
 * [ceil(H/patch)][ceil(W/patch)], packed in view order. */
GSPM_API gspm_status gspm_patch_scale_align(const gspm_views *views, const float *Xr, const float *Xp,
                                   const float *mask, int32_t patch, float *scale_out,
                                   int32_t *count_out, void *stream);

/* Mapping loss of Eq. 17 without the isotropic term, per view k:
 *   L_k = alpha * mean|rgb - rgb_target| + (1 - alpha) * mean|pm - s Xp|
 * with s the per-patch scale of gspm_patch_scale_align computed in the same pass
 * (between pm and Xp, held constant) and means over 3 H W elements.  Writes
 * scale_out as above, loss_out [V] (device, overwritten), and the gradients
 * grad_rgb, grad_pm (packed planes, overwritten; sign(0) = 0).  The context provides
 * scratch for the per-view loss partial sums. */
GSPM_API gspm_status gspm_window_loss(gspm_ctx *ctx, const gspm_views *views, const float *rgb, const float *rgb_target,
                             const float *pm, const float *Xp, int32_t patch, float alpha,
                             float *scale_out, float *loss_out, float *grad_rgb, float *grad_pm,
                             void *stream);

/* Allocation-free gspm_window_loss, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, and harnesses that forbid
 * hipMalloc.  Same arguments, results and kernels as gspm_window_loss, without the
 * context: its per-wave loss partials live in a static device array of
 * GSPM_WINDOW_LOSS_NOALLOC_SLOTS float64 slots (1 MiB) that the library holds on every
 * GPU it runs on until the process ends.  A window needs one slot per strip of
 * floor(64 / patch) horizontally adjacent patches of one patch row, i.e. the sum over its
 * views of ceil(ceil(W / patch) / floor(64 / patch)) * ceil(H / patch) (7,308 for eight
 * keyframes 3x960x640 + 3x1216x352 + 2x640x480 at patch 8; 64,800 for sixteen 1920x1080
 * views); larger windows are rejected with GSPM_ERR_INVALID_ARG before any launch.  The
 * call allocates nothing.  Every slot it reads is written by the same call, so nothing has
 * to start at zero, but the array is shared by all calls on one GPU: calls that overlap
 * on one GPU (on different streams) race and give wrong losses.  The first call on each
 * GPU looks up that GPU's address of the array (hipGetSymbolAddress, no allocation);
 * make that first call outside graph capture. */
#define GSPM_WINDOW_LOSS_NOALLOC_SLOTS 131072
GSPM_API gspm_status gspm_window_loss_noalloc(const gspm_views *views, const float *rgb, const float *rgb_target,
                                              const float *pm, const float *Xp, int32_t patch, float alpha,
                                              float *scale_out, float *loss_out, float *grad_rgb, float *grad_pm,
                                              void *stream);

/* ---- scale alignment and pointmap replacement (supplementary Alg. 1; Sec. 3.3.2, Eq. 14) */

/* Parameters of the patch-based scale alignment (the supplementary parameter table gives
 * P = 10, delta_mu = delta_sigma = 0.3, eps_r = 0.1, max_iter = 3, tau = 0.01). */
typedef struct {
    int32_t patch;      /* P in [2, 64] */
    float delta_mu;     /* patch test |mu_r - mu_p| < delta_mu mu_p */
    float delta_sigma;  /* patch test |sd_r - sd_p| < delta_sigma sd_p */
    float eps_r;        /* correct point |Xr_N - Xp_N| < eps_r */
    int32_t max_iter;   /* iterations, >= 1 */
    float tau;          /* too few correct points: |CP| < tau N_p */
} gspm_align_params;

/* Result per view (device memory). */
typedef struct {
    double scale;          /* sigma': the aligned prior is scale * Xp */
    int32_t cp;            /* correct points of the last iteration */
    int32_t n_valid;       /* N_p: pixels with mask != 0 */
    int32_t insufficient;  /* 1 if cp < tau n_valid (the caller's remedy applies) */
    int32_t pad;
} gspm_align_result;

/* Alg. 1 for every view of the window.  The per-pixel scalar is the norm |X(x)|; patch
 * means and standard deviations (population) are over pixels with mask != 0 (mask NULL =
 * all; border patches partial); correct points are collected afresh in every iteration
 * over the candidate patches, and sigma' = mean|Xr[CP]| / mean|Xp[CP]| measures the
 * original Xp (an empty CP keeps the previous sigma', initially 1).  Xr, Xp: packed
 * camera-frame pointmaps [3][H][W] per view; mask: packed [H][W] or NULL; result: device
 * [V], overwritten.  The context provides scratch (56 bytes per patch).  Returns
 * GSPM_ERR_INVALID_ARG for NULL arrays or parameters out of range, before any launch. */
GSPM_API gspm_status gspm_align_scale(gspm_ctx *ctx, const gspm_views *views, const float *Xr, const float *Xp,
                                      const float *mask, const gspm_align_params *params,
                                      gspm_align_result *result, void *stream);

/* Eq. 14 for every pixel: Xr_hat = Xr where |Xr - s Xp| <= eps_m |s Xp| (s = result[v].scale),
 * else s Xp (products and norms in float64, outputs rounded to float).  Xr_hat may not
 * alias Xr or Xp.  replaced_out: device int32 [V], overwritten with the replaced-pixel
 * count of each view. */
GSPM_API gspm_status gspm_replace_pointmap(const gspm_views *views, const float *Xr, const float *Xp,
                                           const gspm_align_result *result, float eps_m, float *Xr_hat,
                                           int32_t *replaced_out, void *stream);

/* ---- pose initialisation (Sec. 3.2.1, Eq. 6-9) ------------------------------------- */

/* RANSAC + PnP parameters. */
typedef struct {
    int32_t n_hypotheses; /* H: rows of the sample array, >= 1 */
    float threshold;      /* inlier reprojection error in pixels, > 0 */
    int32_t iterations;   /* Gauss-Newton steps per refinement round, >= 0 */
    int32_t rounds;       /* refinement rounds; the inliers are re-selected after each, >= 0 */
} gspm_pnp_params;

/* Relative pose T (frame A -> camera frame B, T_n = T T_ak) from n 2D-3D correspondences:
 * X [3][n] points in frame A (the rendered pointmap of the adjacent keyframe), uv [2][n]
 * pixels of frame B with intrinsics K (host).  samples: device int32 [H][6] indices drawn
 * by the caller (out-of-range rows give invalid hypotheses).  Each hypothesis is the
 * linear six-point PnP on its sample (points centred and scaled, eigenvector of least
 * eigenvalue, det > 0, nearest rotation, mean singular value as the scale); it scores the
 * correspondences with positive depth and reprojection error < threshold; the best (ties
 * to the lowest index) is refined by Gauss-Newton on the squared reprojection errors of its
 * inliers, with T <- Exp(xi) T and damping 1e-9 trace(J^T J) / 6, inliers re-selected
 * after each round.  Outputs (device): T_out float64 [12] row-major [R | t], n_inliers
 * int32 [1], inlier_mask uint8 [n] (may be NULL), scores int32 [H] (may be NULL; -1 for an
 * invalid hypothesis).  With T_ak (device float [12], the adjacent keyframe's world->camera
 * pose) and T_n_out (device float [12]) both non-NULL, the new frame's pose T_n = T T_ak
 * (Eq. 9) is written too.  All arithmetic after the float32 loads is float64.  The context
 * provides scratch (104 bytes per hypothesis and 1 byte per correspondence). */
GSPM_API gspm_status gspm_pnp_ransac(gspm_ctx *ctx, const float *X, const float *uv, int64_t n,
                                     const gspm_intrinsics *K, const int32_t *samples,
                                     const gspm_pnp_params *params, double *T_out, int32_t *n_inliers,
                                     uint8_t *inlier_mask, int32_t *scores, const float *T_ak, float *T_n_out,
                                     void *stream);

/* ---- regulariser and keyframe window (Sec. 3.3.3 Eq. 16; supplementary Eq. S1-S2) -- */

/* Isotropic regulariser of Eq. 16: loss = weight * sum_i sum_k |s_ik - mean_k s_ik| with
 * s = exp(log_scales) (float64 inside; sign(0) = 0).  loss_out: device float [1],
 * overwritten; grad_log_scales: device [3][n], accumulated (+=), may be NULL.  The
 * context provides scratch for the partial sums. */
GSPM_API gspm_status gspm_iso_loss(gspm_ctx *ctx, const gspm_gaussians *g, float weight, float *loss_out,
                                   float *grad_log_scales, void *stream);

/* Covisibility of the views of one forward (supplementary Eq. S1-S2): with G_i the
 * Gaussians that contribute to at least one pixel of view i, iou_out[i][j] =
 * |G_i & G_j| / |G_i | G_j| and oc_out[i][j] = |G_i & G_j| / min(|G_i|, |G_j|) (0 for an
 * empty denominator); count_out[i] = |G_i| (may be NULL).  Device float64 [V][V] and
 * int64 [V], overwritten.  The forward must have run with settings.mark_visible != 0;
 * otherwise the outputs are NaN and count_out is -1.  frame_state and views are those of
 * that forward (n_gaussians its Gaussian count). */
GSPM_API gspm_status gspm_covisibility(gspm_ctx *ctx, const gspm_views *views, int64_t n_gaussians,
                                       const void *frame_state, double *iou_out, double *oc_out,
                                       int64_t *count_out, void *stream);

/* Median of the positive values of each view's depth image (the lower middle value for
 * an even count, 0 for a view without positive depth): the median pointmap depth of the
 * keyframe rule.  depth: packed [H][W] per view; median_out: device float [V]. */
GSPM_API gspm_status gspm_median_depth(gspm_ctx *ctx, const gspm_views *views, const float *depth,
                                       float *median_out, void *stream);

/* T_cw[v] <- Exp(xi[v]) T_cw[v] for every view (device arrays [V][12], [V][6]). */
GSPM_API gspm_status gspm_pose_retract(int32_t n_views, float *T_cw, const float *xi, void *stream);

/* ---- diagnostics -------------------------------------------------------------------- */

/* Launch phases timed by the context when timing is on. */
typedef enum {
    GSPM_PHASE_PREPROCESS = 0, /* projection of every (Gaussian, view) record */
    GSPM_PHASE_DEPTH_SORT = 1, /* radix sort of records by depth */
    GSPM_PHASE_BINNING = 2,    /* pair-count scan, pair emission, range extraction */
    GSPM_PHASE_TILE_SORT = 3,  /* radix sort of tile pairs */
    GSPM_PHASE_RASTER_FWD = 4, /* forward compositing kernel */
    GSPM_PHASE_RASTER_BWD = 5, /* backward compositing kernel */
    GSPM_PHASE_PARAM_BWD = 6,  /* image-plane -> parameter and pose gradients */
    GSPM_PHASE_COUNT = 7
} gspm_phase;

/* Turn per-phase HIP event timing on or off for a context.  While on, each forward and
 * backward records a start/end event pair around every phase on its stream (do not
 * turn it on for calls captured into a graph). */
GSPM_API gspm_status gspm_timing_enable(gspm_ctx *ctx, int32_t on);

/* Wait for the recorded events, add each phase's elapsed milliseconds to ms_out
 * [GSPM_PHASE_COUNT] and its number of timed launches to counts_out (either may be
 * NULL), and forget the recorded events. */
GSPM_API gspm_status gspm_timing_collect(gspm_ctx *ctx, double *ms_out, int64_t *counts_out);

/* Message of the last error on this thread ("" if none). */
GSPM_API const char *gspm_last_error(void);

/* Library version string. */
GSPM_API const char *gspm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GSPM_H */
