// Projective point-to-plane ICP (UPSLAM Section III-B, Equation 1) on gfx950.
//
// One launch = one Gauss-Newton iteration of one pyramid level:
//
//   0. every block reads the block partials left by the previous launch and
//      reduces them in the same fixed order, so every block solves the same
//      6x6 system (Cholesky, FP64) and applies the same update
//      T <- Exp(xi) T (FP64): no atomics, no fences, no extra solve launch --
//      the kernel boundary is the only synchronisation;
//   1. association of K pixels per thread at the new pose: rigid transform,
//      spherical re-projection into the keyframe, the Omega filter, the
//      point-to-plane residual r = (q - s1).n1 and J = [q x n1, n1];
//   2. the 29-value reduction [21 x J^T J | 6 x J^T r | r^2 | inliers]:
//      Kahan-compensated FP32 per thread, then FP64 (or plain FP32 in the
//      FP32 precision mode) quad sums by DPP and the 64 quad sums of each
//      value added through LDS by 8 threads in a fixed order, written as one
//      partial per block.  Partials are stored by value (value v of every
//      block in one row), so that step 0 reads them with coalesced 16-byte
//      loads, 8 threads per value, and issues the state load beside them.
//
// The registration state (pose, status, flags) lives in two ping-pong slots:
// launch n reads slot n%2 and block 0 writes slot (n+1)%2.  Block partials are
// ping-ponged the same way.  A final evaluation launch applies the last update
// and accumulates the quality terms at level 0; a one-block finish launch
// writes the result.
//
// The same kernels serve one registration (descriptor passed by value) and a
// batch of registrations of different sizes (descriptors in device memory,
// block -> (registration, tile) through a per-level prefix table).
#include "ups_icp_kernels.hpp"

namespace ups {

// ------------------------------------------------- pyramid + registration init

// Pyramid of one surfel image from its level-1 pixel q: level-1 pixel (i, j)
// is level-0 pixel (2i, 2j); when i and j are even it is also level-2 pixel
// (i/2, j/2), and level-3 pixel (i/4, j/4) when both are multiples of 4.
__device__ __forceinline__ void pyramid_from_level1(const DGeom *g, const float4 *const *img, int levels, int q) {
    const int W1 = g[1].cols;
    const int i = q / W1, j = q - i * W1;
    const float4 v = ldg(img[0], (2 * i) * g[0].cols + 2 * j);
    ((float4 *)img[1])[q] = v;
    if (levels > 2 && ((i | j) & 1) == 0) ((float4 *)img[2])[(i >> 1) * g[2].cols + (j >> 1)] = v;
    if (levels > 3 && ((i | j) & 3) == 0) ((float4 *)img[3])[(i >> 2) * g[3].cols + (j >> 2)] = v;
}

// Batch: blocks [0, init_blocks) initialise the states from init[k]; the
// other blocks build the pyramids, one thread per level-1 pixel, found
// through the prefix table of per-registration level-1 pixel counts (scan,
// then keyframe).
// With a mask, registrations whose mask byte is 0 are marked to skip the call.
// With need, only the images need[k] names (bit 0 the scan, bit 1 the
// keyframe) are built, and pix_start counts only their level-1 pixels.
__global__ __launch_bounds__(kBlock) void k_prepare_batch(const Inst *__restrict__ insts, const ups_pose *init,
                                                          int n, int levels, int init_blocks,
                                                          const int *__restrict__ pix_start,
                                                          const uint8_t *__restrict__ mask,
                                                          const uint8_t *__restrict__ need) {
    if ((int)blockIdx.x < init_blocks) {
        const int k = blockIdx.x * kBlock + threadIdx.x;
        if (k >= n) return;
        RegState S;
        memset(&S, 0, sizeof(S));
        for (int e = 0; e < 9; e++) S.R[e] = init[k].R[e];
        for (int e = 0; e < 3; e++) S.t[e] = init[k].t[e];
        S.status = UPS_CONVERGED;
        S.level_active = 1;
        S.active = 1;
        if (mask && !mask[k]) {
            S.skip = 1;
            S.stop = 1;
            S.active = 0;
        }
        insts[k].state[0] = S;
        return;
    }
    const int t = (blockIdx.x - init_blocks) * kBlock + threadIdx.x;
    if (t >= pix_start[n]) return;
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pix_start[mid] <= t) lo = mid;
        else hi = mid;
    }
    const Inst &I = insts[lo];
    const int q = t - pix_start[lo];
    const int n0 = (need && !(need[lo] & 1)) ? 0 : I.sg[1].rows * I.sg[1].cols;
    if (q < n0) pyramid_from_level1(I.sg, I.scan, levels, q);
    else pyramid_from_level1(I.kg, I.kf, levels, q - n0);
}

// mask: null = every registration, pyramids built; else only the masked-in
// registrations run and the pyramids of the previous call are reused.  need:
// null = every image's pyramid, else those of the images need[k] names
// (pix_start / total_pix count their level-1 pixels; 0: the states only).
ups_status launch_prepare_batch(const Inst *insts, const ups_pose *init, int n, int levels, const int *pix_start,
                                int total_pix, const uint8_t *mask, const uint8_t *need, hipStream_t s) {
    const int ib = (n + kBlock - 1) / kBlock;
    const int pb = mask ? 0 : (total_pix + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_prepare_batch, dim3(ib + pb), dim3(kBlock), 0, s, insts, init, n, levels, ib, pix_start,
                       mask, need);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

// The pyramids alone (no registration state is touched); with need, those of
// the images need[k] names only (pix_start then counts their pixels).
ups_status launch_build_pyramids(const Inst *insts, int n, int levels, const int *pix_start, int total_pix,
                                 const uint8_t *need, hipStream_t s) {
    const int pb = (total_pix + kBlock - 1) / kBlock;
    if (pb == 0) return UPS_OK;
    hipLaunchKernelGGL(k_prepare_batch, dim3(pb), dim3(kBlock), 0, s, insts, (const ups_pose *)nullptr, n, levels, 0,
                       pix_start, (const uint8_t *)nullptr, need);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

// One block: mask[k] = (inlier ratio of result k < min_ratio), and the
// Compact list of the masked registrations (block-wide prefix sums over
// chunks of 256 registrations, in registration order).
__global__ __launch_bounds__(256) void k_fallback_plan(int n, const ups_icp_result *__restrict__ res,
                                                        double min_ratio, const int *__restrict__ tile_start,
                                                        uint8_t *__restrict__ mask, Compact *__restrict__ hdr,
                                                        int *__restrict__ list, int *__restrict__ start,
                                                        int32_t *__restrict__ count) {
    __shared__ int sc[2][5][256];
    __shared__ int carry[5];
    const int tid = threadIdx.x;
    if (tid < 5) carry[tid] = 0;
    if (tid < 4) start[tid * (n + 1)] = 0;
    __syncthreads();
    for (int c0 = 0; c0 < n; c0 += 256) {
        const int k = c0 + tid;
        int v[5] = {0, 0, 0, 0, 0};
        if (k < n) {
            v[0] = res[k].inlier_ratio < min_ratio ? 1 : 0;
            mask[k] = (uint8_t)v[0];
            if (v[0])
                for (int l = 0; l < 4; l++) v[1 + l] = tile_start[l * (n + 1) + k + 1] - tile_start[l * (n + 1) + k];
        }
        // inclusive Hillis-Steele scans of the five quantities
        int buf = 0;
        for (int q = 0; q < 5; q++) sc[0][q][tid] = v[q];
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            for (int q = 0; q < 5; q++) {
                const int x = sc[buf][q][tid] + (tid >= off ? sc[buf][q][tid - off] : 0);
                sc[buf ^ 1][q][tid] = x;
            }
            buf ^= 1;
            __syncthreads();
        }
        if (v[0]) {
            const int m = carry[0] + sc[buf][0][tid] - 1;
            list[m] = k;
            for (int l = 0; l < 4; l++) start[l * (n + 1) + m + 1] = carry[1 + l] + sc[buf][1 + l][tid];
        }
        __syncthreads();
        if (tid < 5) carry[tid] += sc[buf][tid][255];
        __syncthreads();
    }
    if (tid == 0) {
        hdr->count = carry[0];
        for (int l = 0; l < 4; l++) hdr->total[l] = carry[1 + l];
        if (count) *count = carry[0];
    }
}

// Where the fallback ran and ended with a lower truncated cost, its result
// replaces the first one, marked UPS_FALLBACK_USED.
__global__ void k_fallback_merge(int n, ups_icp_result *__restrict__ res, const ups_icp_result *__restrict__ alt,
                                 const uint8_t *__restrict__ mask) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || !mask[k]) return;
    if (alt[k].trunc_cost < res[k].trunc_cost) {
        res[k] = alt[k];
        res[k].status = UPS_FALLBACK_USED;
    }
}

ups_status launch_fallback_plan(int n, const ups_icp_result *res, double min_ratio, const int *tile_start,
                                uint8_t *mask, Compact *hdr, int *list, int *start, int32_t *count, hipStream_t s) {
    hipLaunchKernelGGL(k_fallback_plan, dim3(1), dim3(256), 0, s, n, res, min_ratio, tile_start, mask, hdr, list,
                       start, count);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_fallback_merge(int n, ups_icp_result *res, const ups_icp_result *alt, const uint8_t *mask,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_fallback_merge, dim3((n + 255) / 256), dim3(256), 0, s, n, res, alt, mask);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

__global__ __launch_bounds__(kBlock) void k_subsample(const float4 *__restrict__ src, int cols0, int level,
                                                      int rows, int cols, float4 *__restrict__ dst) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= rows * cols) return;
    const int i = q / cols, j = q - i * cols;
    dst[q] = src[(size_t)(i << level) * cols0 + (j << level)];
}

ups_status launch_subsample(const DGeom &g0, const float4 *src, int level, float4 *dst, hipStream_t s) {
    const int rows = g0.rows >> level, cols = g0.cols >> level;
    const int n = rows * cols;
    hipLaunchKernelGGL(k_subsample, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, g0.cols, level, rows,
                       cols, dst);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

// -------------------------------------------------------------- launchers

// Pixels per thread for a single registration: as few as keep the block
// count at or below 256, so that step 0 reads at most 256 partials.
int pick_k_single(int npix) {
    int K = 1;
    while (K < 16 && (npix + kBlock * K - 1) / (kBlock * K) > 256) K *= 2;
    return K;
}

// Every registration active at its current pose with no update pending (the
// batch iteration launch timed alone).
__global__ void k_activate_batch(const Inst *__restrict__ insts, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    RegState &S = insts[k].state[0];
    S.active = 1;
    S.level_active = 1;
    S.stop = 0;
    S.pending = 0;
    S.skip = 0;
}

ups_status launch_activate_batch(const Inst *insts, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_activate_batch, dim3((n + 255) / 256), dim3(256), 0, s, insts, n);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_finish_batch_list(int prec, const Inst *insts, const Compact *hdr, const int *list, int blocks,
                                    int parity, ups_icp_result *results, hipStream_t s) {
    UPS_DISPATCH_P(prec, hipLaunchKernelGGL(k_finish_batch_list<PP>, dim3(blocks), dim3(kBlock), 0, s, insts, hdr,
                                            list, parity, results))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_finish_batch(int prec, const Inst *insts, int n, int parity, ups_icp_result *results,
                               hipStream_t s) {
    UPS_DISPATCH_P(prec, hipLaunchKernelGGL(k_finish_batch<PP>, dim3(n), dim3(kBlock), 0, s, insts, parity, results))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

static ups_status launch_finish_one(int prec, const Inst &I, int parity, hipStream_t s) {
    UPS_DISPATCH_P(prec, hipLaunchKernelGGL(k_finish_one<PP>, dim3(1), dim3(kBlock), 0, s, I, parity))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

static ups_status launch_collapse_one(int prec, const Inst &I, int parity, hipStream_t s) {
    UPS_DISPATCH_P(prec, hipLaunchKernelGGL(k_collapse_one<PP>, dim3(1), dim3(kBlock), 0, s, I, parity))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

// One iteration or evaluation launch of a single registration: the variant
// (world frame, IRLS, plain) selects the translation unit that holds it.
static ups_status launch_one(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                             hipStream_t s) {
    if (I.world) {
        if (a.irls_delta > 0.f) {
            set_error("the world-frame variant has no IRLS objective");
            return UPS_ERR_INVALID_ARG;
        }
        return launch_icp_one_world(K, prec, mode, I, a, blocks, s);
    }
    if (a.irls_delta > 0.f) return launch_icp_one_irls(K, prec, mode, I, a, blocks, s);
    return launch_icp_one_plain(K, prec, mode, I, a, blocks, s);
}

// A registration: the Gauss-Newton launches level by level (the first builds
// the state from the start pose; each applies the previous launch's update),
// the evaluation launch and the finish launch that writes the result.  Levels
// are read from the level-0 images (no pyramid copies); the descriptor carries
// the state / partials scratch; pixels per thread follow pick_k_single.
ups_status launch_register(const Inst &I0, const ups_pose *init, const ups_icp_params &p, hipStream_t s) {
    Inst I = I0;
    int Ks[4] = {1, 1, 1, 1};
    for (int l = 0; l < p.levels; l++) {
        const int npix = I.sg[l].rows * I.sg[l].cols;
        Ks[l] = pick_k_single(npix);
        I.nblocks[l] = (npix + kBlock * Ks[l] - 1) / (kBlock * Ks[l]);
    }
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.cos_theta = p.cos_theta_max;
    a.irls_delta = p.irls_delta;
    a.min_inliers = p.min_inliers;
    a.stop_norm = p.stop_update_norm;
    a.init = init;
    int parity = 0;
    ups_status st;
    a.prev_level = -1;
    for (int l = p.levels - 1; l >= 0; l--) {
        a.level = l;
        a.d_max2 = p.d_max[l] * p.d_max[l];
        // a level small enough for one XCD runs all its iterations in one launch
        // (the launches after it, at least the evaluation, zero its counters)
        if (p.iters[l] >= 2 && I.xsync && I.nblocks[l] <= kLevelXcdMaxTiles && Ks[l] <= 2 &&
            (a.irls_delta <= 0.f || (!I.world && p.precision == UPS_PREC_KAHAN_F64))) {
            a.parity = parity;
            a.first_of_level = 1;
            if ((st = launch_icp_level_xcd(Ks[l], p.precision, I, a, p.iters[l], I.nblocks[l], s)) != UPS_OK)
                return st;
            a.seq += p.iters[l];
            a.init = nullptr;
            a.prev_level = l;
            parity ^= p.iters[l] & 1;
            continue;
        }
        for (int it = 0; it < p.iters[l]; it++) {
            a.parity = parity;
            a.first_of_level = it == 0;
            if ((st = launch_one(Ks[l], p.precision, MODE_ITER, I, a, I.nblocks[l], s)) != UPS_OK) return st;
            a.seq++;
            a.init = nullptr;
            a.prev_level = l;
            parity ^= 1;
            if (I.nblocks[l] > 256 && (st = launch_collapse_one(p.precision, I, parity, s)) != UPS_OK)
                return st;
        }
    }
    // evaluation at level 0: apply the last update, quality terms; result
    a.level = 0;
    a.parity = parity;
    a.first_of_level = 0;
    a.d_max2 = p.d_max[0] * p.d_max[0];
    a.tau2 = a.d_max2;
    a.check_max_iters = (p.stop_update_norm > 0.0 && p.iters[0] > 0);
    if ((st = launch_one(Ks[0], p.precision, MODE_EVAL, I, a, I.nblocks[0], s)) != UPS_OK) return st;
    return launch_finish_one(p.precision, I, parity ^ 1, s);
}

// Normal equations at a fixed pose: one evaluation launch that builds the
// state from the pose, then the finish launch that writes the totals.
ups_status launch_eval(const Inst &I0, const ups_pose *T, float d_max, float cos_theta, int precision,
                       hipStream_t s) {
    Inst I = I0;
    const int npix = I.sg[0].rows * I.sg[0].cols;
    const int K = pick_k_single(npix);
    I.nblocks[0] = (npix + kBlock * K - 1) / (kBlock * K);
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.level = 0;
    a.parity = 0;
    a.prev_level = -1;
    a.d_max2 = d_max * d_max;
    a.tau2 = a.d_max2;
    a.cos_theta = cos_theta;
    a.init = T;
    const ups_status st = launch_one(K, precision, MODE_EVAL, I, a, I.nblocks[0], s);
    if (st != UPS_OK) return st;
    return launch_finish_one(precision, I, 1, s);
}

// ---------------------------------------------------------- correspondences

__global__ __launch_bounds__(kBlock) void k_correspondences(DGeom sg, const float4 *__restrict__ scan, DGeom kg,
                                                            const float4 *__restrict__ kf, const ups_pose *pose,
                                                            float d_max2, float cos_theta, int32_t *idx,
                                                            uint8_t *inl) {
    const int npix = sg.rows * sg.cols;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const Rt32 T = load_pose_f32(pose);
    const int i = p / sg.cols, j = p - i * sg.cols;
    const Pair pr = associate(sg, scan[p], i, j, kg, kf, T, d_max2, cos_theta);
    idx[p] = pr.kf_index;
    inl[p] = pr.inlier ? 1 : 0;
}

// The world-frame variant at the pose T (scan -> keyframe): the scan's world
// pose world_kf * T is formed in FP64 and both poses are rounded to FP32, as
// the world-frame registration does.
__global__ __launch_bounds__(kBlock) void k_correspondences_world(DGeom sg, const float4 *__restrict__ scan, DGeom kg,
                                                                  const float4 *__restrict__ kf, const ups_pose *pose,
                                                                  ups_pose world_kf, float d_max2, float cos_theta,
                                                                  int32_t *idx, uint8_t *inl) {
    const int npix = sg.rows * sg.cols;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    Rt32 T, W;
    for (int a = 0; a < 3; a++) {
        for (int c = 0; c < 3; c++)
            T.r[3 * a + c] = (float)(world_kf.R[3 * a] * pose->R[c] + world_kf.R[3 * a + 1] * pose->R[3 + c] +
                                     world_kf.R[3 * a + 2] * pose->R[6 + c]);
        T.t[a] = (float)(world_kf.R[3 * a] * pose->t[0] + world_kf.R[3 * a + 1] * pose->t[1] +
                         world_kf.R[3 * a + 2] * pose->t[2] + world_kf.t[a]);
    }
    for (int k = 0; k < 9; k++) W.r[k] = (float)world_kf.R[k];
    for (int k = 0; k < 3; k++) W.t[k] = (float)world_kf.t[k];
    const int i = p / sg.cols, j = p - i * sg.cols;
    const Gather G = scan_side_world(sg, scan[p], ldg(sg.lut_row, i * sg.stride), ldg(sg.lut_col, j * sg.stride), kg,
                                     kf, T, W);
    bool in;
    float r;
    float3 n1;
    kf_side_world(kg, G, W, d_max2, cos_theta, in, r, n1);
    idx[p] = G.kf_index;
    inl[p] = in ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_project_points(DGeom g, const float *__restrict__ xyz, int64_t n,
                                                           int32_t *ii, int32_t *jj) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const float3 q = make_float3(xyz[3 * k], xyz[3 * k + 1], xyz[3 * k + 2]);
    int i = -1, j = -1;
    if (!project(g, q, i, j)) i = j = -1;
    ii[k] = i;
    jj[k] = j;
}

ups_status launch_project_points(const DGeom &g, const float *xyz, int64_t n, int32_t *ii, int32_t *jj,
                                 hipStream_t s) {
    if (n == 0) return UPS_OK;
    hipLaunchKernelGGL(k_project_points, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, g, xyz, n,
                       ii, jj);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_correspondences_world(const DGeom &sg, const float4 *scan, const DGeom &kg, const float4 *kf,
                                        const ups_pose *T, const ups_pose &world_kf, float d_max, float cos_theta,
                                        int32_t *idx, uint8_t *inl, hipStream_t s) {
    const int npix = sg.rows * sg.cols;
    hipLaunchKernelGGL(k_correspondences_world, dim3((npix + kBlock - 1) / kBlock), dim3(kBlock), 0, s, sg, scan, kg,
                       kf, T, world_kf, d_max * d_max, cos_theta, idx, inl);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_correspondences(const DGeom &sg, const float4 *scan, const DGeom &kg, const float4 *kf,
                                  const ups_pose *T, float d_max, float cos_theta, int32_t *idx, uint8_t *inl,
                                  hipStream_t s) {
    const int npix = sg.rows * sg.cols;
    hipLaunchKernelGGL(k_correspondences, dim3((npix + kBlock - 1) / kBlock), dim3(kBlock), 0, s, sg, scan, kg, kf,
                       T, d_max * d_max, cos_theta, idx, inl);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
