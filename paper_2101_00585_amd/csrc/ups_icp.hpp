// Registration descriptors shared by the single and batched ICP launchers.
#pragma once

#include "ups_internal.hpp"

namespace ups {

// MODE_SCHED: an iteration tile of the persistent batch kernel (the
// iteration sums; state and partial exchanged as agent-coherent words).
enum { MODE_ITER = 0, MODE_EVAL = 1, MODE_SCHED = 2 };

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

// One registration as the kernels see it.  Batches read pyramid images of
// each level (scan[l], kf[l]); single registrations (the fused kernels) read
// level l straight from the level-0 images, every 2^l-th row and column.
struct Inst {
    DGeom sg[4], kg[4];           // geometry of each pyramid level
    const float4 *scan[4], *kf[4];  // surfel images of each level (level 0 = caller's)
    RegState *state;              // [2]
    double *partials;             // [2][kPartialStride][pstride]: value v of block b at [v * pstride + b]
    int pstride;                  // a multiple of 16
    int nblocks[4];               // blocks (tiles) per level
    ups_icp_result *res;          // finish target (or null)
    ups_normal_eq *neq;           // finish target (or null)
    unsigned int *xsync;          // single registrations: [4][2] ticket and arrival counters of the one-XCD level
                                  // kernel per level (zero between calls; later launches reset them), or null
    // world-frame variant: the state pose is the scan's world pose, wR/wt the
    // keyframe's; init and result stay scan -> keyframe
    int world;
    double wR[9], wt[3];
};

// Scratch of a single registration (128-byte aligned): two state slots, then,
// on a cache line of their own, the one-XCD level kernels' counters, a pair
// per level (zero between calls).
constexpr size_t kXsyncOffset = (2 * sizeof(RegState) + 127) / 128 * 128;
constexpr size_t kSingleStateBytes = kXsyncOffset + 128;
inline unsigned int *xsync_of(RegState *state) { return (unsigned int *)((char *)state + kXsyncOffset); }
// Tiles of a level the one-XCD level kernel takes (they must all be resident
// on one XCD's 32 CUs at once).
constexpr int kLevelXcdMaxTiles = 32;
// Unsuccessful polls of a waiting workgroup of the level kernel, in all, after
// which it gives up and the registration ends as DEGENERATE; the setting of
// later launches (ups_debug_level_spin_limit).
constexpr unsigned kLevelSpinLimit = 1u << 21;
unsigned level_spin_limit();

// Per-launch arguments.
struct StepArgs {
    int level, parity, first_of_level, check_max_iters;
    int prev_level;  // level of the previous launch (-1: none), whose partials this launch reduces
    float d_max2, cos_theta, tau2;
    float irls_delta;  // > 0: inlier terms weighted by 1 / max(|r|, irls_delta)
    int min_inliers;
    double stop_norm;
    int kpt;  // MODE_SCHED: pixels per thread of this tile (<= the kernel's K, a multiple of its pixel groups)
    const ups_pose *init;  // single registrations: the first launch builds the state from this start pose
    int reverse_tiles;  // debug: workgroups take the tiles in reverse order (set by the launchers)
    int seq;            // single registrations: the launch's number within the call (phase timestamps)
    // batches: (registration << 16) | tile of each of the level's tiles in tile
    // order (null: found by binary search in the prefix table of tile counts)
    const unsigned *tile_of;
};

// Debug tile order of the iteration / evaluation launches (ups_debug_reverse_tile_order).
bool debug_reverse_tiles();
inline StepArgs with_tile_order(const StepArgs &a) {
    StepArgs b = a;
    b.reverse_tiles = debug_reverse_tiles() ? 1 : 0;
    return b;
}

// A subset of a batch's registrations: list[m] for m < count, and per level
// l the prefix table start[l][m] (m <= count) of their tile counts, whose
// total is total[l].  Device memory: header, then list[n], then start[4][n+1].
struct Compact {
    int count;
    int total[4];
};

// Persistent batch scheduler (k_icp_persistent): the registrations of a
// batch call advance independently through one launch.  A job is one
// Gauss-Newton iteration of one registration: its
// tiles are published under consecutive ticket numbers; workers take tickets
// in order, process the tile, and the last tile of a job to finish reduces
// the job's partials, updates the registration and publishes its next job.
struct SchedJob {
    int level, mode, iter, ntiles;  // pyramid level, MODE_ITER (MODE_EVAL: done), iteration within the level, tiles
};

struct Sched {
    unsigned int next_ticket;  // tickets handed out
    unsigned int published;    // tickets that carry a tile
    int outstanding;           // registrations whose iterations have not finished
    int error;                 // 1: a worker stopped waiting (spin limit): the call's results are incomplete
    unsigned int epoch;        // call number; tile-map entries of this call carry it
    int pad[3];
};

struct SchedArgs {
    Sched *sched;
    unsigned long long *tile_map;  // [map_size]: (epoch << 32) | (registration << 10) | tile
    SchedJob *jobs;                // [n]: the job in flight of each registration
    int *arrived;                  // [n]: its tiles finished so far
    const Inst *insts;             // [n]
    ups_icp_result *results;       // [n]
    const uint8_t *mask;           // [n] or null: registrations taking part (k_sched_init)
    int n, map_size, levels;
    int kpt[4];                    // pixels per thread of a tile at each level (<= the kernel's K)
    int iters[4];
    float d_max2[4];
    float cos_theta, irls_delta;
    int min_inliers;
    double stop_norm;
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
                                 const uint8_t *need, hipStream_t s);
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
// fused: the batch's main loop (each block applies its registration's pending
// update, state and partials in the ping-pong slots of a.parity); otherwise the
// pose is in state slot 0.
ups_status launch_icp_batch(int K, int prec, int mode, const Inst *insts, const int *tile_start, int n,
                            const StepArgs &a, int blocks, hipStream_t s, bool fused = false);
ups_status launch_icp_batch_fused(int K, int prec, int mode, const Inst *insts, const int *tile_start, int n,
                                  const StepArgs &a, int blocks, hipStream_t s);
ups_status launch_icp_one_plain(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                                hipStream_t s);
ups_status launch_icp_one_world(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                                hipStream_t s);
ups_status launch_icp_one_irls(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                               hipStream_t s);
// All `iters` Gauss-Newton iterations of level a.level of a single
// registration in one launch whose tiles all run on one XCD (see
// k_icp_level_xcd); `tiles` = I.nblocks[a.level].
ups_status launch_icp_level_xcd(int K, int prec, const Inst &I, const StepArgs &a, int iters, int tiles,
                                hipStream_t s);
ups_status launch_icp_batch_irls(int K, int prec, int mode, const Inst *insts, const int *tile_start, int n,
                                 const StepArgs &a, int blocks, hipStream_t s, bool fused);
ups_status launch_icp_batch_list_irls(int K, int prec, int mode, const Inst *insts, const Compact *hdr,
                                      const int *list, const int *start_l, int n, const StepArgs &a, int blocks,
                                      hipStream_t s);
ups_status launch_activate_batch(const Inst *insts, int n, hipStream_t s);
// Scheduler set-up (first jobs of the registrations taking part) and the
// persistent launch (grid = resident blocks of the kernel).
ups_status launch_sched_init(const SchedArgs &A, hipStream_t s);
ups_status launch_icp_persistent(int K, int prec, const SchedArgs &A, int blocks, hipStream_t s);
// Resident blocks of the persistent kernel for (K, prec, IRLS) on the current device.
int persistent_grid(int K, int prec, bool irls);
// pixels per thread the persistent kernel is instantiated for
bool persistent_k_supported(int K);
// The results of the listed registrations (state slot `parity`).
ups_status launch_finish_batch_list(int prec, const Inst *insts, const Compact *hdr, const int *list, int blocks,
                                    int parity, ups_icp_result *results, hipStream_t s);
ups_status launch_finish_batch(int prec, const Inst *insts, int n, int parity, ups_icp_result *results,
                               hipStream_t s);
ups_status launch_prepare_batch(const Inst *insts, const ups_pose *init, int n, int levels, const int *pix_start,
                                int total_pix, const uint8_t *mask, const uint8_t *need, hipStream_t s);
ups_status launch_fallback_plan(int n, const ups_icp_result *res, double min_ratio, const int *tile_start,
                                uint8_t *mask, Compact *hdr, int *list, int *start, int32_t *count, hipStream_t s);
ups_status launch_icp_batch_list(int K, int prec, int mode, const Inst *insts, const Compact *hdr, const int *list,
                                 const int *start_l, int n, const StepArgs &a, int blocks, hipStream_t s);
ups_status launch_fallback_merge(int n, ups_icp_result *res, const ups_icp_result *alt, const uint8_t *mask,
                                 hipStream_t s);
__device__ __host__ inline int npartials_host(int nblocks) { return nblocks > 256 ? 1 : nblocks; }

}  // namespace ups
