/*
 * upslam.h -- C ABI of the MI355X (gfx950) projective-ICP registration library.
 *
 * The library implements the data-parallel hot path of UPSLAM (Cowley, Miller,
 * Taylor, "UPSLAM: Union of Panoramas SLAM", arXiv 2101.00585):
 *   - surface normals of a panoramic range image          (Section III-A)
 *   - registration of a sweep against a keyframe by ICP   (Section III-B, Eq. 1)
 *     with the point-to-plane metric over projective correspondences and the
 *     similarity filter Omega_{d,theta}
 *   - the count-weighted keyframe update                  (Section III-C)
 *
 * Conventions for every call
 *   - Device pointers are caller-owned (e.g. torch tensors), 16-byte aligned for
 *     float4 images, and never freed or retained by the library.
 *   - Every call is asynchronous on the given HIP stream (a hipStream_t passed as
 *     void*; NULL = the default stream).  Results land in device memory; the
 *     caller synchronises before reading them.  Device memory is allocated only
 *     by ups_context_create (per-registration scratch), ups_batch_create (a
 *     batch's scratch) and ups_autotune (its measurement buffers);
 *     ups_register_scan / ups_fuse_scan / ups_panorama_normals /
 *     ups_batch_normals / ups_register_batch enqueue only kernels, so they can
 *     be captured into a HIP graph (geometries must have been seen once outside
 *     capture, see ups_context_create).
 *   - One context holds the scratch space of one registration at a time: calls
 *     on the same context must be ordered (same stream, or synchronised).
 *   - A non-zero return is a usage or HIP error (message in ups_last_error()).
 *     Numerical outcomes are not errors: they are reported in
 *     ups_icp_result.status.
 *
 * Panorama layout: a range image is float[rows][cols] (row-major).  Row i looks
 * along elevation el_top - i*d_el, column j along azimuth 2*pi*j/cols (column 0
 * along +x, counter-clockwise about +z); the ray is (cos el cos az, cos el sin
 * az, sin el) and the point is range * ray.  A range is valid iff finite and
 * r_min < r <= r_max (compared in FP32).  A surfel image is
 * float[rows][cols][4] = (nx, ny, nz, range): range 0 = no return, normal
 * (0,0,0) = no normal.  Keyframe sample counts are uint16[rows][cols].
 * A pose is T = (R, t), FP64, R row-major, mapping scan coordinates into
 * keyframe coordinates: x_kf = R x_scan + t (the T of Equation 1, s1 in the
 * keyframe, s2 in the sweep).
 */
#ifndef UPSLAM_H
#define UPSLAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    UPS_OK = 0,
    UPS_ERR_INVALID_ARG = -1, /* bad pointer, size, geometry or parameter */
    UPS_ERR_HIP = -2,         /* a HIP runtime call failed */
    UPS_ERR_UNSUPPORTED = -3, /* valid request the library does not support */
    UPS_ERR_WORKSPACE = -4    /* request exceeds what the context was created for */
} ups_status;

/* ups_icp_result.status values */
enum {
    UPS_CONVERGED = 0,     /* finished: stop criterion met, or fixed iteration count done */
    UPS_MAX_ITERS = 1,     /* stop criterion > 0 was not met at level 0 */
    UPS_DEGENERATE = 2,    /* J^T J not positive definite: pose left at the last good value */
    UPS_NO_INLIERS = 3,    /* fewer than min_inliers correspondences: pose left unchanged */
    UPS_FALLBACK_USED = 4  /* batch: proposal rejected, identity-initialised result kept */
};

/* ups_icp_params.precision values */
enum {
    UPS_PREC_KAHAN_F64 = 0, /* FP32 per pixel; per-thread FP32 sums, Kahan-compensated for J^T r,
                               sum r^2 and the truncated cost (plain for J^T J); FP64 cross-lane,
                               block and grid sums, FP64 solve and pose update */
    UPS_PREC_F32 = 1,       /* FP32 everywhere, including the solve and the pose update */
    UPS_PREC_F64 = 2        /* FP32 per pixel, per-thread sums of the (exact) FP64 products in FP64,
                               FP64 beyond: on gfx950 an FP64 FMA issues at the FP32 rate, so this
                               is cheaper than the compensated FP32 sums and more accurate */
};

typedef struct {
    int32_t rows, cols;
    double el_top, d_el; /* radians */
    double r_min, r_max; /* metres */
} ups_geom;

typedef struct {
    double R[9]; /* row-major */
    double t[3];
} ups_pose;

/* Normal estimation (Section III-A).  The raw normal of pixel (i, j) is the
 * normalised cross product of the vectors from its point to the points of
 * (i, j+1 mod cols) and (i+1, j) -- (i-1, j) on the last row -- oriented towards
 * the sensor.  No normal when a range is invalid, when a neighbour's range
 * differs by more than max_rel_jump * r, or when the cross product is
 * degenerate.  Then atrous_levels passes of an edge-aware a-trous filter: 5x5
 * B3-spline taps spaced 2^l, weights exp(-((r_q-r_p)/(sigma_r r_p))^2) *
 * exp(-(2-2 n_p.n_q)/sigma_n^2), renormalised.  Defaults: 2, 0.5, 0.05, 0.5. */
typedef struct {
    int32_t atrous_levels;
    float sigma_n, sigma_r, max_rel_jump;
} ups_normal_params;

/* Registration (Section III-B).  Coarse-to-fine over `levels` (1..4) pyramid
 * levels (level l keeps every 2^l-th row and column); iters[l] Gauss-Newton
 * steps at level l on the squared point-to-plane residuals of Equation 1, or,
 * with irls_delta > 0, on Equation 1's absolute residuals by iteratively
 * reweighted least squares: each inlier's terms carry the weight
 * 1 / max(|r|, irls_delta) (the fixed point minimises Huber's function with
 * that threshold, |r| - irls_delta/2 above it).  irls_delta = 0: squared
 * objective, bit-identical to the unweighted path.
 * Omega: inlier iff both surfels are valid, |q - s1| <= d_max[l] and
 * (R n2).n1 >= cos_theta_max.  A level ends early when stop_update_norm > 0 and
 * the step norm |xi| falls below it.  min_inliers: fewer correspondences stop
 * the registration with UPS_NO_INLIERS.  rows and cols must be divisible by
 * 2^(levels-1) and cols/2^(levels-1) by 64. */
typedef struct {
    int32_t levels;
    int32_t iters[4];
    float d_max[4];
    float cos_theta_max;
    double stop_update_norm;
    int32_t min_inliers;
    int32_t precision; /* UPS_PREC_* */
    float irls_delta;  /* 0: squared residuals; >= 1e-6: absolute residuals by IRLS (metres) */
} ups_icp_params;

/* Result of a registration (device memory).  T: final pose.  The quality block
 * is evaluated at level 0 and the final pose (Section III-C): inliers over
 * valid scan ranges, rms of inlier residuals, truncated cost sum over valid
 * scan pixels of min(r^2, d_max[0]^2) with non-inliers counting d_max[0]^2, and
 * the normal equations (upper triangle of J^T J row-major, J^T r) there, with
 * the IRLS weights when irls_delta > 0 (the quality terms are unweighted). */
typedef struct {
    ups_pose T;
    double rms, trunc_cost, inlier_ratio;
    int64_t inliers, valid;
    int32_t iters_run, status;
    int32_t level_iters[4]; /* updates applied at each pyramid level */
    double JtJ[21], Jtr[6];
    double last_update_norm;
} ups_icp_result;

/* Normal equations at a fixed pose (device memory), see ups_normal_equations. */
typedef struct {
    double JtJ[21], Jtr[6];
    double sum_r2;
    int64_t inliers, valid;
} ups_normal_eq;

/* Keyframe update (Section III-C): keyframe pixels holding c > 0 samples take a
 * sample from the registered sweep if it passes |q - s1| <= d_max,
 * m.n1 >= cos_theta_max and |u.n1| >= min_cos_incidence; range and normal are
 * averaged with weights c : 1 and c <- min(c+1, max_count).  Empty keyframe
 * pixels take the nearest (smallest |q|, then smallest scan index) scan surfel
 * projecting onto them, with c = 1. */
typedef struct {
    float d_max, cos_theta_max, min_cos_incidence;
    int32_t max_count;
} ups_fuse_params;

typedef struct ups_context ups_context;

/* Create a context on `device` for panoramas of up to max_pixels pixels and
 * batches of up to max_batch registrations whose panoramas total at most
 * max_batch_pixels pixels (scan and keyframe each).  The scratch of single
 * registrations, normals and fusion (a-trous buffer, fill keys, block
 * partials, state, ray tables) is allocated here; a batch allocates its
 * own in ups_batch_create.  The first use of a new panorama geometry
 * uploads its ray tables synchronously; such a first use is rejected during
 * stream capture (UPS_ERR_INVALID_ARG). */
ups_status ups_context_create(ups_context **out, int device, int64_t max_pixels, int32_t max_batch,
                              int64_t max_batch_pixels);
void ups_context_destroy(ups_context *ctx);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *ups_last_error(void);

/* Debug (determinism checks, Section III-B reductions): with reversed != 0,
 * every registration iteration / evaluation launch enqueued afterwards, in any
 * thread, deals its tiles to workgroups in the reverse of the usual order.
 * Block partials are reduced in tile order, so results are bitwise the same
 * either way.  Process-wide; launches already enqueued or captured keep the
 * order they were enqueued with.  Always UPS_OK. */
ups_status ups_debug_reverse_tile_order(int32_t reversed);

/* Debug (failure handling of the one-XCD level kernel, which runs all
 * Gauss-Newton iterations of a coarse pyramid level of a single registration,
 * Section III-B, in one launch whose workgroups wait for each other between
 * iterations): a waiting workgroup of a level kernel enqueued afterwards gives
 * up after `polls` unsuccessful polls in all (0: at its first) and the
 * registration ends as UPS_DEGENERATE; the launch still ends.  polls < 0
 * restores the default, 2^21.  Process-wide; launches already enqueued or
 * captured keep their limit.  UPS_ERR_INVALID_ARG if polls >= 2^32. */
ups_status ups_debug_level_spin_limit(int64_t polls);

/* Surfel image (Section III-A) from a range image.  depth_d: float[rows][cols];
 * surfel_d: float[rows][cols][4] output (must not alias depth_d). */
ups_status ups_panorama_normals(ups_context *ctx, const ups_geom *g, const float *depth_d, float *surfel_d,
                                const ups_normal_params *p, void *stream);

/* Pyramid level `level` (>= 1) of a surfel image: pixel (i, j) = level-0 pixel
 * (2^l i, 2^l j).  out_d: float[rows>>l][cols>>l][4]. */
ups_status ups_pyramid_level(ups_context *ctx, const ups_geom *g, const float *surfel_d, int32_t level,
                             float *out_d, void *stream);

/* Register a sweep's surfel image against a keyframe's surfel image
 * (Section III-B).  init_d: device pose to start from (may alias
 * &result_d->T).  result_d: device ups_icp_result written by the call. */
ups_status ups_register_scan(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                             const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *init_d,
                             const ups_icp_params *p, ups_icp_result *result_d, void *stream);

/* ups_register_scan for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * no context, no allocation.  Same arguments (minus the context), numerics,
 * result and errors as ups_register_scan; it runs on the calling thread's
 * current device, and `stream` (NULL = the default stream) must belong to it.
 * Its scratch (both panoramas' ray tables, the block partials and the
 * registration state, 0.82 MB) is a static array in device memory
 * that each GPU holds from the library's first use until the process ends;
 * scan and keyframe are limited to 262144 pixels each (e.g. 128 x 2048):
 * larger ones return UPS_ERR_WORKSPACE.  All calls on one GPU share that
 * array: calls that overlap in time on one GPU (different streams or
 * threads) race and must be ordered by the caller.  Enqueues only kernels. */
ups_status ups_register_scan_noalloc(const ups_geom *scan_g, const float *scan_surfel_d, const ups_geom *kf_g,
                                     const float *kf_surfel_d, const ups_pose *init_d, const ups_icp_params *p,
                                     ups_icp_result *result_d, void *stream);

/* Fuse a registered sweep into a keyframe in place (Section III-C).  T_d: device
 * pose scan -> keyframe (e.g. &result_d->T).  kf_surfel_d / kf_count_d are
 * read and written; the sweep's surfel image is only read. */
ups_status ups_fuse_scan(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                         const ups_geom *kf_g, float *kf_surfel_d, uint16_t *kf_count_d, const ups_pose *T_d,
                         const ups_fuse_params *p, void *stream);

/* Panorama formation (Section III-A): the measurements of one sweep, each
 * taken in the frame of its own firing instant, are moved into the frame of a
 * single instant and projected into a panoramic image that keeps the nearest
 * return per pixel.  A valid range r at (i, j) of raw_g (row = beam, column =
 * firing) gives x = r u(i, j) and y = C_j x; y lands on its pixel of out_g
 * when |y| is a valid range of out_g, and the smallest |y| wins (the smaller
 * measurement index among equal FP32 ranges).
 *   raw_range_d  device float [raw rows][raw cols], 0 = no return;
 *   col_T_d      device float [raw cols][12]: C_j as R (row-major) then t,
 *                column j's frame -> the reference frame (e.g. the
 *                gyroscope's rotations, t = 0), or NULL for the identity;
 *   depth_d      device float [out rows][out cols], written (0 = empty);
 *                out_g may differ from raw_g (a wider keyframe field of view).
 * Uses the context's fill scratch (out rows * cols <= max_pixels): calls on
 * one context must not overlap in time.  Two kernels on `stream`. */
ups_status ups_splat_sweep(ups_context *ctx, const ups_geom *raw_g, const float *raw_range_d, const float *col_T_d,
                           const ups_geom *out_g, float *depth_d, void *stream);

/* ---- keyframe management (Section III-C) -------------------------------- */

/* Moving-object check between two keyframes, run when the current keyframe
 * changes: the keyframes together record which space was seen empty, so a
 * sample of one that the other looked through belongs to something that
 * moved.  A sample of keyframe A (valid range r at pixel (i, j), point
 * x = r u(i, j)) is removed when, with y = T_ba x projected to B's pixel
 * (i', j'), every pixel of B's 3x3 neighbourhood of (i', j') (columns wrap; a
 * neighbourhood that leaves B's rows keeps the sample) holds a valid range
 * exceeding |y| + max(margin_abs, margin_rel |y|) with at least min_count
 * fused samples (b_count_d NULL: any count).  Mutual when b_mask_d is given:
 * B's samples are tested against A with T_ba^-1, both from the unmodified
 * images, then the marked samples of both are removed.
 *   T_ba_d      device pose mapping A's frame into B's;
 *   a/b_surfel  device float4 [rows][cols] surfel images, modified in place:
 *               removed samples become (0, 0, 0, 0);
 *   a/b_count   device uint16 [rows][cols] sample counts (may be NULL),
 *               removed samples get count 0;
 *   a/b_mask    caller-owned uint8 [rows][cols] outputs, 1 = removed;
 *               b_mask_d NULL: only A is tested and modified;
 *   removed_d   device int32 [2] (may be NULL): numbers removed from A and B.
 * Enqueues three kernels on `stream`; the images must not alias. */
typedef struct {
    float margin_abs, margin_rel; /* metres, fraction of the range */
    int32_t min_count;            /* samples a voting pixel needs */
} ups_consistency_params;

ups_status ups_keyframe_consistency(ups_context *ctx, const ups_geom *a_g, float *a_surfel_d, uint16_t *a_count_d,
                                    const ups_geom *b_g, float *b_surfel_d, uint16_t *b_count_d,
                                    const ups_pose *T_ba_d, const ups_consistency_params *p, uint8_t *a_mask_d,
                                    uint8_t *b_mask_d, int32_t *removed_d, void *stream);

/* Loop-closure classes (Section III-C) for n registrations of the current
 * scan against neighbouring keyframes (results_d, device): STRONG when the
 * inlier ratio exceeds new_keyframe_ratio (the quality below which a new
 * keyframe is sought; the neighbour becomes the current keyframe), WEAK when
 * it exceeds 3/4 of it (a pose-graph edge only), NONE otherwise and for
 * registrations that ended UPS_DEGENERATE or UPS_NO_INLIERS.  class_d: device
 * int32 [n]; best_d (device int32, may be NULL): the STRONG closure with the
 * highest ratio, the lowest index among equals, -1 when there is none.  One
 * kernel on `stream`. */
enum { UPS_LOOP_NONE = 0, UPS_LOOP_WEAK = 1, UPS_LOOP_STRONG = 2 };
ups_status ups_classify_loop_closures(ups_context *ctx, int32_t n, const ups_icp_result *results_d,
                                      double new_keyframe_ratio, int32_t *class_d, int32_t *best_d, void *stream);

/* Projective correspondences at a fixed pose at level 0 (Section III-B):
 * kf_index_d[rows*cols] = keyframe pixel index i*cols+j the scan point projects
 * to, or -1 (no scan surfel or outside the keyframe's rows); inlier_d = 1 iff
 * the pair passes Omega with thresholds d_max / cos_theta_max. */
ups_status ups_correspondences(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                               const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *T_d, float d_max,
                               float cos_theta_max, int32_t *kf_index_d, uint8_t *inlier_d, void *stream);

/* ------------------------------------------------------------------------
 * Precision study: world-frame coordinates.  The keyframe-frame calls above
 * never form world coordinates, so a keyframe's distance from the world
 * origin (the 4.4 km drive of Section IV-F) cannot reach
 * their FP32 arithmetic.  These two variants carry every point in world
 * coordinates in FP32 instead, given the keyframe's world pose, to measure
 * what that costs.  Same arguments, layout and errors as their keyframe-frame
 * counterparts; init, T and the result pose stay scan -> keyframe.
 * ------------------------------------------------------------------------ */

/* ups_register_scan with the Gauss-Newton state held as the scan's world pose
 * world_kf_h * T (FP64); per iteration the scan's and the keyframe's world
 * poses are rounded to FP32, scan points and keyframe surfels are taken to
 * world coordinates, the scan point is re-expressed in the keyframe frame only
 * to find its pixel, and the residual r = (q - s1).n1 and J = [q x n1, n1] are
 * formed from world coordinates (the update is a left perturbation of the
 * world pose).  world_kf_h: host pointer, finite. */
ups_status ups_register_scan_world(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                                   const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *world_kf_h,
                                   const ups_pose *init_d, const ups_icp_params *p, ups_icp_result *result_d,
                                   void *stream);

/* ups_correspondences with the association of ups_register_scan_world. */
ups_status ups_correspondences_world(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                                     const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *world_kf_h,
                                     const ups_pose *T_d, float d_max, float cos_theta_max, int32_t *kf_index_d,
                                     uint8_t *inlier_d, void *stream);

/* Spherical projection (the lookup behind the projective correspondences of
 * Section III-B): for each of n points xyz_d[n][3] (FP32, the panorama's
 * sensor frame) the nearest pixel centre, i_d[k] = row and j_d[k] = column,
 * or -1 / -1 for the origin and for directions outside the panorama's rows. */
ups_status ups_project_points(ups_context *ctx, const ups_geom *g, const float *xyz_d, int64_t n, int32_t *i_d,
                              int32_t *j_d, void *stream);

/* Gauss-Newton normal equations of Equation 1 at a fixed pose at level 0, with
 * the given precision mode's reduction (UPS_PREC_*). */
ups_status ups_normal_equations(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                                const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *T_d, float d_max,
                                float cos_theta_max, int32_t precision, ups_normal_eq *out_d, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many independent registrations of uneven panorama sizes (e.g. the
 * candidate transforms of a loop-closure search, Section III-C) advanced
 * together.  Two schedulers, chosen per batch (ups_batch_set_scheduler):
 *   UPS_SCHED_LAUNCHES (default): one launch per Gauss-Newton iteration covers
 *     every registration of the batch, each block first applying its
 *     registration's update from the previous launch's sums; a registration
 *     that met its stop criterion or failed drops out of the remaining
 *     launches (its blocks exit at once).
 *   UPS_SCHED_PERSISTENT: one persistent launch in which each registration
 *     advances through its iterations as its own chain of jobs (the tiles of
 *     an iteration, then the update by the block that finishes the last
 *     tile), so the launch's work follows the active registrations.
 * Both end with one evaluation launch over all registrations at their final
 * poses and one finish launch, give the same results (the same fixed-order
 * sums), and are fixed at planning time, so a whole ups_register_batch call
 * can be captured in a HIP graph.
 * ------------------------------------------------------------------------ */

/* One registration of a batch.  scan_surfel_d / kf_surfel_d are the surfel
 * images the registration reads; when scan_depth_d / kf_depth_d are not NULL,
 * ups_batch_normals writes the surfel images from them. */
typedef struct {
    ups_geom scan_g, kf_g;
    const float *scan_depth_d, *kf_depth_d;
    float *scan_surfel_d, *kf_surfel_d;
} ups_batch_item;

typedef struct ups_batch ups_batch;

/* Plan a batch of n registrations sharing the parameters p: validates the
 * items, uploads their descriptors and allocates the batch's scratch
 * (pyramids, states, partials).  Synchronous; not for use during capture.
 * pixels_per_thread: a power of two up to 64, or 0 for the library's choice
 * (the autotuned value for these sizes if ups_autotune has run).  n is at
 * most the context's max_batch and 65535.  Every item must satisfy the
 * ups_register_scan constraints and have at most 256 * 256 * 64 pixels, and
 * an item with depth at most 8191 normal tiles of 64 x 16 pixels. */
ups_status ups_batch_create(ups_context *ctx, int32_t n, const ups_batch_item *items_h, const ups_icp_params *p,
                            int32_t pixels_per_thread, ups_batch **out);
void ups_batch_destroy(ups_batch *b);

/* Surfel images (Section III-A) of every item that has depth pointers, one
 * launch per a-trous level over all of them (in UPS_PYR_IN_NORMALS mode also
 * the batch's pyramids, see ups_batch_set_pyramid_mode). */
ups_status ups_batch_normals(ups_context *ctx, ups_batch *b, const ups_normal_params *p, void *stream);

/* Run every registration of the batch from init_d[n] (device poses) and write
 * results_d[n] (device).  Same numerics as ups_register_scan. */
ups_status ups_register_batch(ups_context *ctx, ups_batch *b, const ups_pose *init_d, ups_icp_result *results_d,
                              void *stream);

/* Fallback of proposal-started registrations (the learned proposal below):
 * call right after ups_register_batch on the same batch with its results.
 * Registrations whose inlier ratio is below min_inlier_ratio are registered
 * again from the identity (with the pyramids of that call); where the second
 * run ends with a lower truncated cost its result replaces the first in
 * results_d, with status UPS_FALLBACK_USED.  The others are not run again.
 * Enqueues only kernels (graph-capturable). */
ups_status ups_register_batch_fallback(ups_context *ctx, ups_batch *b, double min_inlier_ratio,
                                       ups_icp_result *results_d, void *stream);

/* The two halves of ups_register_batch_fallback, for callers that skip the
 * second when nothing needs it (its launch sequence has a fixed cost even
 * when empty): plan flags the registrations to rerun and writes their number
 * to count_d (device int32, may be NULL); run reruns the flagged ones of the
 * last plan and merges their results into results_d. */
ups_status ups_batch_fallback_plan(ups_context *ctx, ups_batch *b, double min_inlier_ratio,
                                   const ups_icp_result *results_d, int32_t *count_d, void *stream);
ups_status ups_batch_fallback_run(ups_context *ctx, ups_batch *b, ups_icp_result *results_d, void *stream);

/* Loop-closure grid search (Section III-C): for every registration k of the
 * batch, score the candidate transforms base_d[k] * G_c by a coarse projective
 * alignment test -- the number of Omega inliers (thresholds
 * d_max, cos_theta_max) of the scan's pyramid level `level` against the
 * keyframe's -- and write the best candidate (most inliers, the lowest c among
 * equals) to best_d[k] and its score to best_score_d[k] (may be NULL).
 * Candidates c = (a * n_xy + u) * n_xy + v for a < n_yaw, u, v < n_xy:
 * G_c = (Rz(2 pi a / n_yaw), ((u - h) xy_step, (v - h) xy_step, 0)),
 * h = (n_xy - 1) / 2.  scores_d: caller-owned int32 [n][C] workspace, C =
 * n_yaw n_xy^2 <= 65535, left holding every candidate's score.  Builds the
 * batch's pyramids from the level-0 surfel images first; enqueues only
 * kernels.  The best poses can start ups_register_batch. */
typedef struct {
    int32_t level;
    int32_t n_yaw, n_xy;
    float xy_step;
    float d_max, cos_theta_max;
} ups_grid_params;

ups_status ups_batch_grid_search(ups_context *ctx, ups_batch *b, const ups_grid_params *p, const ups_pose *base_d,
                                  int32_t *scores_d, ups_pose *best_d, int32_t *best_score_d, void *stream);

/* Autotune the pixels per thread of batch launches for this device: times the
 * Gauss-Newton launch at 1, 2, 4, ..., 64 pixels per thread on synthetic
 * batches of each lidar panorama size (16x128 ... 128x2048) and keeps the
 * fastest per size in the context for later ups_batch_create calls.  With a
 * cache path, a cache written for the same GPU architecture is loaded instead
 * of measuring, and a fresh measurement is written there as JSON.
 * Synchronous; allocates temporary device memory. */
ups_status ups_autotune(ups_context *ctx, const char *cache_json_path);

/* Time the batch's Gauss-Newton launch at pyramid level `level` alone: marks
 * every registration active at its current pose (no update pending), enqueues n_launches
 * back-to-back launches of that kernel between two HIP events on `stream`, and
 * returns their average duration in microseconds (synchronises the stream).
 * Leaves the registration states unusable for anything but a new
 * ups_register_batch call. */
ups_status ups_batch_time_iteration(ups_context *ctx, ups_batch *b, int32_t level, int32_t n_launches,
                                    void *stream, float *us_per_launch);

/* Pixels per thread the batch launches use at each pyramid level. */
ups_status ups_batch_pixels_per_thread(const ups_batch *b, int32_t out[4]);

enum {
    UPS_SCHED_LAUNCHES = 0,   /* one launch per iteration (default) */
    UPS_SCHED_PERSISTENT = 1  /* one persistent launch, per-registration job chains */
};

/* Choose the scheduler of later ups_register_batch / fallback calls on this
 * batch (UPS_SCHED_*; UPS_ERR_INVALID_ARG otherwise).  Host only; takes
 * effect for calls enqueued afterwards. */
ups_status ups_batch_set_scheduler(ups_batch *b, int32_t scheduler);

enum {
    UPS_PYR_IN_REGISTER = 0, /* ups_register_batch builds the pyramids (default) */
    UPS_PYR_IN_NORMALS = 1   /* ups_batch_normals builds them */
};

/* Where the batch's pyramid levels 1 and up (subsampled copies of every scan
 * and keyframe surfel image that the coarse Gauss-Newton levels read) are
 * built.  UPS_PYR_IN_REGISTER (default): every ups_register_batch and
 * ups_batch_grid_search call builds them from the level-0 surfel images.
 * UPS_PYR_IN_NORMALS: the last a-trous pass of ups_batch_normals also writes
 * the pyramid levels of every image it computes (the items' images with
 * depth), and register and grid-search calls build only those of the other
 * images (surfel images the batch reads as they are, such as resident
 * keyframes): call ups_batch_normals after any change to the depth of an
 * item.  The results are the same either way.  UPS_ERR_INVALID_ARG for
 * another mode.  Host only; takes effect for calls enqueued afterwards. */
ups_status ups_batch_set_pyramid_mode(ups_batch *b, int32_t mode);

/* Gauss-Newton iterations per pyramid level of later ups_register_batch calls
 * on this batch (Section III-B's coarse-to-fine schedule; a start already
 * close to the answer, such as a learned proposal, can leave out the coarsest
 * levels): iters[l] for l < the batch's levels, each in [0, the value the
 * batch was created with]; 0 skips the level.  The fallback calls keep the
 * schedule the batch was created with.  UPS_ERR_INVALID_ARG otherwise.  Host
 * only; takes effect for calls enqueued afterwards. */
ups_status ups_batch_set_iterations(ups_batch *b, const int32_t iters[4]);

/* The persistent launch of UPS_SCHED_PERSISTENT: its blocks (the kernel's
 * resident blocks on the device), and the pixels per thread of a tile at each
 * pyramid level. */
ups_status ups_batch_schedule(const ups_batch *b, int32_t *blocks, int32_t kpt[4]);

/* ------------------------------------------------------------------------
 * Learned pose proposal.  The paper starts loop-closure registrations from a
 * grid search over candidate transforms (Section III-C); this library can
 * instead start a registration from the pose a small convolutional network
 * proposes from the two panoramas, keeping identity-started ICP as the
 * fallback.  The network is the library's own (not in the paper):
 *
 *   input   x[n][32][256][2] bfloat16, NHWC: channel 0 keyframe, 1 scan,
 *           1/range of pixel (y rows/32, x cols/256), 0 where there is no
 *           valid return;
 *   layers  five 3x3 convolutions with ReLU, width circular, height
 *           zero-padded, (cin, cout, stride) = (2,32,2) (32,64,2) (64,96,2)
 *           (96,128,2) (128,128,1), BF16 operands on the matrix cores with
 *           FP32 accumulation, activations stored as bfloat16; then a fully
 *           connected FP32 layer 4096 -> 6 over the NHWC flattening;
 *   output  y[n][6]: the scan -> keyframe pose (Exp(0.25 y[0:3]), 1.0 y[3:6])
 *           (rotation vector in rad, translation in m);
 *   params  FP32, flattened per layer: conv W [9 cin][cout] (row
 *           (3 ky + kx) cin + ci), conv b [cout], ..., FC W [6][4096], FC b [6];
 *   loss    sum of squared output errors / (2 n); optimiser Adam with
 *           beta1 = 0.9, beta2 = 0.999, eps = 1e-8.
 * ------------------------------------------------------------------------ */

#define UPS_PROPOSAL_ROWS 32
#define UPS_PROPOSAL_COLS 256

typedef struct ups_proposal ups_proposal;

/* A range image the network input is taken from: range of pixel (i, j) at
 * range_d[(i * cols + j) * stride] (stride 1 for a depth image; a surfel
 * image's range channel is surfel_d + 3 with stride 4).  rows and cols must be
 * multiples of 32 and 256; a range is valid iff finite and r_min < r <= r_max. */
typedef struct {
    const float *range_d;
    int32_t rows, cols, stride;
    float r_min, r_max;
} ups_range_image;

/* Number of network parameters (357382). */
int64_t ups_proposal_num_params(void);

/* A proposal network for batches of up to max_batch pairs on the context's
 * device: parameters (zero), Adam state, activations and workspace.  Synchronous;
 * allocates device memory. */
ups_status ups_proposal_create(ups_context *ctx, int32_t max_batch, ups_proposal **out);
void ups_proposal_destroy(ups_proposal *p);

/* Host <-> device parameter copies (synchronous).  set_params also resets the
 * Adam moments and step count. */
ups_status ups_proposal_set_params(ups_proposal *p, const float *params_h, int64_t n);
ups_status ups_proposal_get_params(ups_proposal *p, float *params_h, int64_t n);

/* The parameters to / from a file: the 8 bytes "UPSPRM01", the parameter
 * count (little-endian int64, ups_proposal_num_params()), then the FP32
 * parameters.  load rejects any other content with UPS_ERR_INVALID_ARG and,
 * like set_params, resets the Adam moments.  Synchronous. */
ups_status ups_proposal_save(ups_proposal *p, const char *path);
ups_status ups_proposal_load(ups_proposal *p, const char *path);
/* Gradient of the last training step. */
ups_status ups_proposal_get_grads(ups_proposal *p, float *grads_h, int64_t n);

/* Resumable training state to / from a file: the 8 bytes "UPSCKP01", the
 * parameter count and the Adam step count (little-endian int64), then the
 * FP32 parameters, first moments and second moments.  A training step after
 * load_checkpoint continues exactly as it would have after save_checkpoint
 * (the caller keeps its own data order and random state).  load rejects any
 * other content with UPS_ERR_INVALID_ARG and leaves the network unchanged.
 * Synchronous. */
ups_status ups_proposal_save_checkpoint(ups_proposal *p, const char *path);
ups_status ups_proposal_load_checkpoint(ups_proposal *p, const char *path);

/* Diagnostics: the stored output of convolution layer `layer` (1..5, NHWC,
 * bfloat16 bits) for the first n pairs of the last forward pass or training
 * step (act_h), and its gradient dL/dy (FP32) from the last training step
 * (dact_h); either may be NULL.  Host buffers; synchronous. */
ups_status ups_proposal_activations(ups_proposal *p, int32_t layer, int32_t n, uint16_t *act_h, float *dact_h);

/* Record the n (keyframe, scan) image pairs ups_proposal_input reads
 * (synchronous upload of n descriptors; the images must stay alive). */
ups_status ups_proposal_plan_input(ups_proposal *p, int32_t n, const ups_range_image *kf_h,
                                   const ups_range_image *scan_h);

/* Network input of the planned pairs into x_d[n][32][256][2] (bfloat16 bits),
 * or into the proposal's own input buffer when x_d is NULL. */
ups_status ups_proposal_input(ups_proposal *p, uint16_t *x_d, void *stream);

/* y_d[n][6] from x_d (NULL: the proposal's own input buffer). */
ups_status ups_proposal_forward(ups_proposal *p, int32_t n, const uint16_t *x_d, float *y_d, void *stream);

/* poses_d[n] (FP64, scan -> keyframe) from network outputs y_d[n][6]. */
ups_status ups_proposal_poses(ups_proposal *p, int32_t n, const float *y_d, ups_pose *poses_d, void *stream);

/* One Adam step on the batch (x_d, target_d[n][6]) with learning rate lr:
 * forward, loss, backward, update.  loss_d (device float, may be NULL)
 * receives the batch loss before the update. */
ups_status ups_proposal_train_step(ups_proposal *p, int32_t n, const uint16_t *x_d, const float *target_d, float lr,
                                   float *loss_d, void *stream);

/* The network's convolution as separate passes, for any shape (cout a
 * multiple of 4 in [4, 65536], 1 <= cin <= 65536, stride 1 or 2, width a
 * multiple of the stride; otherwise UPS_ERR_INVALID_ARG).  NHWC tensors;
 * x, y bfloat16 bits; dy, dx, dw, db FP32.  Device pointers: x and the
 * weights 8-byte aligned, and in the backward-data pass y 8-byte and dy
 * 16-byte aligned (the kernels load four elements at a time); the others
 * aligned to their element size (UPS_ERR_INVALID_ARG otherwise).
 *   forward:          y = relu(conv(x, W) + b), W given as w_nk[cout][9 cin]
 *                     (the transpose of the [9 cin][cout] layout), bfloat16;
 *   backward (data):  dx = dL/dx from y and dy = dL/dy, W as w_kn[9 cin][cout];
 *   backward (wgt):   dw[9 cin][cout] and db[cout] from x, y, dy, with a
 *                     workspace of ups_conv3x3_backward_weight_work() floats. */
ups_status ups_conv3x3_forward(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t stride,
                               const uint16_t *x_d, const uint16_t *w_nk_d, const float *b_d, uint16_t *y_d,
                               void *stream);
ups_status ups_conv3x3_backward_data(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t stride,
                                     const uint16_t *y_d, const float *dy_d, const uint16_t *w_kn_d, float *dx_d,
                                     void *stream);
int64_t ups_conv3x3_backward_weight_work(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t stride);
ups_status ups_conv3x3_backward_weight(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t stride,
                                       const uint16_t *x_d, const uint16_t *y_d, const float *dy_d, float *dw_d,
                                       float *db_d, float *work_d, int64_t work_floats, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* UPSLAM_H */
