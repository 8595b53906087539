// Keyframe management on the GPU (UPSLAM Section III-C): the moving-object
// check between two keyframes at a keyframe switch, and the classification
// of loop-closure registrations into strong and weak closures.
//
// Moving-object check.  The keyframes together describe which space was
// seen empty: a sample of keyframe A that keyframe B looked through (B's
// rays around the sample's pixel in B all return from farther away, by a
// margin) belongs to something that moved, and is removed.  One launch marks
// both directions from the unmodified images (blocks [0, na) test A's pixels
// against B, the rest B's against A); a second launch removes the marked
// samples.  Two launches, so that no image is cleared while the other
// direction still reads it.
#include "ups_internal.hpp"

namespace ups {

namespace {

struct FreeSpaceJob {
    DGeom src, dst;                // the tested keyframe, the one that votes
    const float4 *src_s, *dst_s;   // their surfel images
    const uint16_t *dst_count;     // votes need dst_count >= min_count (null: any)
    uint8_t *mask;                 // src pixels marked (1) or kept (0)
    float4 *clear_s;               // removal: the src image and counts
    uint16_t *clear_count;
    int inverse;                   // 0: map by T_ba, 1: by its inverse
    int blocks;
};

struct FreeSpaceArgs {
    FreeSpaceJob job[2];
    int njobs;
    float margin_abs, margin_rel;
    int min_count;
    const ups_pose *T_ba;
    int *removed;                  // [2] or null
};

constexpr int kKfBlock = 256;

// T_ba (FP64) or its inverse (R^T, -R^T t) rounded to FP32.
__device__ Rt32 pose_for(const ups_pose *T, int inverse) {
    Rt32 o;
    if (!inverse) {
        for (int k = 0; k < 9; k++) o.r[k] = (float)T->R[k];
        for (int k = 0; k < 3; k++) o.t[k] = (float)T->t[k];
        return o;
    }
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) o.r[3 * a + c] = (float)T->R[3 * c + a];
    for (int a = 0; a < 3; a++)
        o.t[a] = (float)(-(T->R[a] * T->t[0] + T->R[3 + a] * T->t[1] + T->R[6 + a] * T->t[2]));
    return o;
}

__global__ __launch_bounds__(kKfBlock) void k_free_space_mark(FreeSpaceArgs a) {
    __shared__ float Ts[12];
    const int jb = (a.njobs > 1 && (int)blockIdx.x >= a.job[0].blocks) ? 1 : 0;
    const FreeSpaceJob &J = a.job[jb];
    const int blk = blockIdx.x - (jb ? a.job[0].blocks : 0);
    if (threadIdx.x == 0) {
        const Rt32 T = pose_for(a.T_ba, J.inverse);
        for (int k = 0; k < 9; k++) Ts[k] = T.r[k];
        for (int k = 0; k < 3; k++) Ts[9 + k] = T.t[k];
    }
    __syncthreads();
    const int npix = J.src.rows * J.src.cols;
    const int px = blk * kKfBlock + threadIdx.x;
    if (px >= npix) return;
    Rt32 T;
#pragma unroll
    for (int k = 0; k < 9; k++) T.r[k] = Ts[k];
#pragma unroll
    for (int k = 0; k < 3; k++) T.t[k] = Ts[9 + k];
    uint8_t marked = 0;
    const float r = J.src_s[px].w;
    if (range_ok(J.src, r)) {
        const int i = px / J.src.cols, j = px - i * J.src.cols;
        const float3 u = ray(J.src, i, j);
        const float3 y = transform(T, make_float3(r * u.x, r * u.y, r * u.z));
        int bi, bj;
        if (project(J.dst, y, bi, bj) && bi >= 1 && bi + 1 < J.dst.rows) {
            const float rho = __builtin_amdgcn_sqrtf(y.x * y.x + y.y * y.y + y.z * y.z);
            const float thr = rho + fmaxf(a.margin_abs, a.margin_rel * rho);
            const float *dst_r = reinterpret_cast<const float *>(J.dst_s) + 3;
            bool seen = true;
#pragma unroll
            for (int di = -1; di <= 1; di++) {
#pragma unroll
                for (int dj = -1; dj <= 1; dj++) {
                    int jj = bj + dj;
                    jj = jj < 0 ? jj + J.dst.cols : (jj >= J.dst.cols ? jj - J.dst.cols : jj);
                    const int q = (bi + di) * J.dst.cols + jj;
                    const float rb = dst_r[4 * q];
                    const bool votes = J.dst_count == nullptr || (int)J.dst_count[q] >= a.min_count;
                    seen = seen & range_ok(J.dst, rb) & votes & (rb > thr);
                }
            }
            marked = seen ? 1 : 0;
        }
    }
    J.mask[px] = marked;
}

__global__ __launch_bounds__(kKfBlock) void k_remove_marked(FreeSpaceArgs a) {
    __shared__ int block_removed;
    const int jb = (a.njobs > 1 && (int)blockIdx.x >= a.job[0].blocks) ? 1 : 0;
    const FreeSpaceJob &J = a.job[jb];
    const int blk = blockIdx.x - (jb ? a.job[0].blocks : 0);
    if (threadIdx.x == 0) block_removed = 0;
    __syncthreads();
    const int npix = J.src.rows * J.src.cols;
    const int px = blk * kKfBlock + threadIdx.x;
    if (px < npix && J.mask[px]) {
        J.clear_s[px] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (J.clear_count) J.clear_count[px] = 0;
        atomicAdd(&block_removed, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0 && a.removed && block_removed) atomicAdd(&a.removed[jb], block_removed);
}

__global__ void k_zero_pair(int *p) {
    if (threadIdx.x < 2) p[threadIdx.x] = 0;
}

// Loop-closure classes (Section III-C): strong when the registration's
// inlier ratio exceeds the new-keyframe threshold, weak when it exceeds 3/4
// of it, none otherwise or when the registration failed.  best: the strong
// closure with the highest ratio (lowest index among equals), -1 if none.
__global__ __launch_bounds__(256) void k_classify(int n, const ups_icp_result *__restrict__ res, double threshold,
                                                  int32_t *__restrict__ cls, int32_t *__restrict__ best) {
    __shared__ double br[256];
    __shared__ int bk[256];
    const int tid = threadIdx.x;
    double my_r = -1.0;
    int my_k = -1;
    for (int k = tid; k < n; k += 256) {
        const ups_icp_result &R = res[k];
        const bool ok = R.status == UPS_CONVERGED || R.status == UPS_MAX_ITERS || R.status == UPS_FALLBACK_USED;
        const double q = R.inlier_ratio;
        const int c = !ok ? UPS_LOOP_NONE
                          : (q > threshold ? UPS_LOOP_STRONG : (q > 0.75 * threshold ? UPS_LOOP_WEAK : UPS_LOOP_NONE));
        cls[k] = c;
        if (c == UPS_LOOP_STRONG && q > my_r) {  // k increases: the first of equals stays
            my_r = q;
            my_k = k;
        }
    }
    br[tid] = my_r;
    bk[tid] = my_k;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            const double r2 = br[tid + w];
            const int k2 = bk[tid + w];
            if (k2 >= 0 && (bk[tid] < 0 || r2 > br[tid] || (r2 == br[tid] && k2 < bk[tid]))) {
                br[tid] = r2;
                bk[tid] = k2;
            }
        }
        __syncthreads();
    }
    if (tid == 0 && best) *best = bk[0];
}

}  // namespace

}  // namespace ups

using namespace ups;

extern "C" {

ups_status ups_keyframe_consistency(ups_context *ctx, const ups_geom *a_g, float *a_surfel_d, uint16_t *a_count_d,
                                    const ups_geom *b_g, float *b_surfel_d, uint16_t *b_count_d,
                                    const ups_pose *T_ba_d, const ups_consistency_params *p, uint8_t *a_mask_d,
                                    uint8_t *b_mask_d, int32_t *removed_d, void *stream) {
    UPS_REQUIRE(ctx && p, "context / params is null");
    ups_status st;
    if ((st = check_ptr(a_surfel_d, 16, "keyframe A surfel")) != UPS_OK) return st;
    if ((st = check_ptr(b_surfel_d, 16, "keyframe B surfel")) != UPS_OK) return st;
    if ((st = check_ptr(T_ba_d, 8, "pose")) != UPS_OK) return st;
    if ((st = check_ptr(a_mask_d, 1, "mask A")) != UPS_OK) return st;
    if (a_count_d && (st = check_ptr(a_count_d, 2, "count A")) != UPS_OK) return st;
    if (b_count_d && (st = check_ptr(b_count_d, 2, "count B")) != UPS_OK) return st;
    if (b_mask_d && (st = check_ptr(b_mask_d, 1, "mask B")) != UPS_OK) return st;
    if (removed_d && (st = check_ptr(removed_d, 4, "removed")) != UPS_OK) return st;
    UPS_REQUIRE(std::isfinite(p->margin_abs) && std::isfinite(p->margin_rel) && p->margin_abs >= 0.f &&
                    p->margin_rel >= 0.f && p->min_count >= 0 && p->min_count <= 65535,
                "invalid consistency params");
    UPS_REQUIRE((const void *)a_surfel_d != (const void *)b_surfel_d, "the two keyframes must not alias");
    UPS_REQUIRE(b_mask_d == nullptr || (const void *)a_mask_d != (const void *)b_mask_d,
                "the two masks must not alias");
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    hipStream_t s = (hipStream_t)stream;
    DGeom ga, gb;
    if ((st = device_geom(ctx, a_g, 0, s, &ga)) != UPS_OK) return st;
    if ((st = device_geom(ctx, b_g, 0, s, &gb)) != UPS_OK) return st;
    FreeSpaceArgs a;
    memset(&a, 0, sizeof(a));
    a.margin_abs = p->margin_abs;
    a.margin_rel = p->margin_rel;
    a.min_count = p->min_count;
    a.T_ba = T_ba_d;
    a.removed = removed_d;
    const int na = (a_g->rows * a_g->cols + kKfBlock - 1) / kKfBlock;
    const int nb = (b_g->rows * b_g->cols + kKfBlock - 1) / kKfBlock;
    a.job[0] = FreeSpaceJob{ga, gb, (const float4 *)a_surfel_d, (const float4 *)b_surfel_d, b_count_d, a_mask_d,
                            (float4 *)a_surfel_d, a_count_d, 0, na};
    a.njobs = 1;
    if (b_mask_d) {
        a.job[1] = FreeSpaceJob{gb, ga, (const float4 *)b_surfel_d, (const float4 *)a_surfel_d, a_count_d, b_mask_d,
                                (float4 *)b_surfel_d, b_count_d, 1, nb};
        a.njobs = 2;
    }
    const int blocks = na + (b_mask_d ? nb : 0);
    if (removed_d) {
        hipLaunchKernelGGL(k_zero_pair, dim3(1), dim3(64), 0, s, removed_d);
        UPS_CHECK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_free_space_mark, dim3(blocks), dim3(kKfBlock), 0, s, a);
    UPS_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_remove_marked, dim3(blocks), dim3(kKfBlock), 0, s, a);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status ups_classify_loop_closures(ups_context *ctx, int32_t n, const ups_icp_result *results_d,
                                      double new_keyframe_ratio, int32_t *class_d, int32_t *best_d, void *stream) {
    UPS_REQUIRE(ctx, "context is null");
    UPS_REQUIRE(n >= 1 && n <= (1 << 24), "n must be in [1, 2^24]");
    UPS_REQUIRE(std::isfinite(new_keyframe_ratio), "new_keyframe_ratio must be finite");
    ups_status st;
    if ((st = check_ptr(results_d, 8, "results")) != UPS_OK) return st;
    if ((st = check_ptr(class_d, 4, "class")) != UPS_OK) return st;
    if (best_d && (st = check_ptr(best_d, 4, "best")) != UPS_OK) return st;
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    hipLaunchKernelGGL(k_classify, dim3(1), dim3(256), 0, (hipStream_t)stream, n, results_d, new_keyframe_ratio,
                       class_d, best_d);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // extern "C"
