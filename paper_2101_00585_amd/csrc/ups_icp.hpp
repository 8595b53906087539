// Registration descriptors shared by the single and batched ICP launchers.
#pragma once

#include "ups_internal.hpp"

namespace ups {

enum { MODE_ITER = 0, MODE_EVAL = 1 };

// Registration state, two ping-pong slots per registration.
struct RegState {
    double R[9], t[3];  // current pose (scan -> keyframe)
    double last_norm;   // |xi| of the last applied update
    int iters_run;      // applied updates
    int status;         // UPS_CONVERGED / UPS_MAX_ITERS / UPS_DEGENERATE / UPS_NO_INLIERS
    int stop;           // the registration stopped (degenerate / too few inliers)
    int level_active;   // 0 once the current level met its stop criterion
    int pending;        // the partials of the previous launch await their update
    int npartials;      // number of those partials
    int level_iters[4]; // updates applied per level
    int active;         // batches: the next Gauss-Newton launch processes this registration
    int skip;           // batches: the registration takes no part in this call (masked out)
};

// One registration as the kernels see it.
struct Inst {
    DGeom sg[4], kg[4];           // geometry of each pyramid level
    const float4 *scan[4], *kf[4];  // surfel images of each level (level 0 = caller's)
    RegState *state;              // [2]
    double *partials;             // [2][kPartialStride][pstride]: value v of block b at [v * pstride + b]
    int pstride;                  // a multiple of 16
    int nblocks[4];               // blocks (tiles) per level
    ups_icp_result *res;          // finish target (or null)
    ups_normal_eq *neq;           // finish target (or null)
    // world-frame variant: the state pose is the scan's world pose, wR/wt the
    // keyframe's; init and result stay scan -> keyframe
    int world;
    double wR[9], wt[3];
};

// Per-launch arguments.
struct StepArgs {
    int level, parity, first_of_level, check_max_iters;
    int prev_level;  // level of the previous launch (-1: none), whose partials this launch reduces
    float d_max2, cos_theta, tau2;
    float irls_delta;  // > 0: inlier terms weighted by 1 / max(|r|, irls_delta)
    int min_inliers;
    double stop_norm;
};

// A subset of a batch's registrations: list[m] for m < count, and per level
// l the prefix table start[l][m] (m <= count) of their tile counts, whose
// total is total[l].  Device memory: header, then list[n], then start[4][n+1].
struct Compact {
    int count;
    int total[4];
};

// Loop-closure grid search over candidate transforms (see ups_grid.hip).
struct GridArgs {
    int level, n_yaw, n_xy, C;
    float xy_step, d_max2, cos_theta;
};

int pick_k_single(int npix);
ups_status launch_grid_search(const Inst *insts, const int *tile_start_l, int n, int K, int tiles,
                              const ups_pose *base, const GridArgs &g, int *scores, ups_pose *best, int *best_score,
                              hipStream_t s);
ups_status launch_build_pyramids(const Inst *insts, int n, int levels, const int *pix_start, int total_pix,
                                 hipStream_t s);
ups_status launch_register(const Inst &I, const ups_pose *init, const ups_icp_params &p, hipStream_t s);
ups_status launch_correspondences_world(const DGeom &sg, const float4 *scan, const DGeom &kg, const float4 *kf,
                                        const ups_pose *T, const ups_pose &world_kf, float d_max, float cos_theta,
                                        int32_t *idx, uint8_t *inl, hipStream_t s);
ups_status launch_eval(const Inst &I, const ups_pose *T, float d_max, float cos_theta, int precision,
                       hipStream_t s);
// Iteration / evaluation launches of the ICP kernel.  Batches pick the IRLS
// instantiation themselves when a.irls_delta > 0; single registrations go
// through launch_register / launch_eval.  Each variant lives in its own
// translation unit (ups_icp_iter_*.hip).
ups_status launch_icp_batch(int K, int prec, int mode, const Inst *insts, const int *tile_start, int n,
                            const StepArgs &a, int blocks, hipStream_t s);
ups_status launch_icp_one_plain(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                                hipStream_t s);
ups_status launch_icp_one_world(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                                hipStream_t s);
ups_status launch_icp_one_irls(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                               hipStream_t s);
ups_status launch_icp_batch_irls(int K, int prec, int mode, const Inst *insts, const int *tile_start, int n,
                                 const StepArgs &a, int blocks, hipStream_t s);
ups_status launch_icp_batch_list_irls(int K, int prec, int mode, const Inst *insts, const Compact *hdr,
                                      const int *list, const int *start_l, int n, const StepArgs &a, int blocks,
                                      hipStream_t s);
ups_status launch_activate_batch(const Inst *insts, int n, hipStream_t s);
ups_status launch_solve_batch(int prec, const Inst *insts, int n, const StepArgs &a, hipStream_t s);
ups_status launch_solve_batch_list(int prec, const Inst *insts, const Compact *hdr, const int *list, int blocks,
                                   const StepArgs &a, hipStream_t s);
ups_status launch_finish_batch(int prec, const Inst *insts, int n, int parity, ups_icp_result *results,
                               hipStream_t s);
ups_status launch_prepare_batch(const Inst *insts, const ups_pose *init, int n, int levels, const int *pix_start,
                                int total_pix, const uint8_t *mask, hipStream_t s);
ups_status launch_fallback_plan(int n, const ups_icp_result *res, double min_ratio, const int *tile_start,
                                uint8_t *mask, Compact *hdr, int *list, int *start, int32_t *count, hipStream_t s);
ups_status launch_icp_batch_list(int K, int prec, int mode, const Inst *insts, const Compact *hdr, const int *list,
                                 const int *start_l, int n, const StepArgs &a, int blocks, hipStream_t s);
ups_status launch_fallback_merge(int n, ups_icp_result *res, const ups_icp_result *alt, const uint8_t *mask,
                                 hipStream_t s);
__device__ __host__ inline int npartials_host(int nblocks) { return nblocks > 256 ? 1 : nblocks; }

}  // namespace ups
