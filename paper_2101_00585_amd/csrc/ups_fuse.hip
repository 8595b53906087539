// Keyframe update (UPSLAM Section III-C) on gfx950.
//
//   k_fuse_update_fill  one launch, two kinds of blocks:
//     update blocks, one thread per keyframe pixel: pixels holding samples
//       are mapped back into the sweep (T^-1), gated by the similarity filter
//       and averaged with weights count : 1;
//     fill blocks, one thread per sweep pixel: valid surfels are projected
//       into the keyframe and compete for its empty pixels with a 64-bit
//       atomicMin on (FP32 bits of |q|, sweep index) -- the nearest surface
//       wins, ties broken by the smaller index.
//   k_fuse_resolve  one thread per keyframe pixel: winners are written with
//     count 1 and their fill key is reset.
// Update and fill touch disjoint keyframe pixels (count > 0 vs count == 0 at
// entry; an update keeps count > 0), so they can run in the same launch.  The
// fill keys are all-ones between calls: set at context creation, restored by
// the resolve pass.
#include "ups_internal.hpp"

namespace ups {

struct FuseArgs {
    DGeom sg, kg;
    const float4 *scan;
    float4 *kf;
    uint16_t *count;
    unsigned long long *key;
    const ups_pose *pose;
    float d_max2, cos_theta, min_cos_inc;
    int max_count;
};

constexpr unsigned long long kNoKey = ~0ull;

__device__ __forceinline__ void fuse_update(const FuseArgs &a, int px) {
    // no FMA contraction: a sample at the pixel's own point must give r_new = r
#pragma clang fp contract(off)
    const int npix = a.kg.rows * a.kg.cols;
    if (px >= npix) return;
    const int c = a.count[px];
    if (c == 0) return;
    const float4 s1 = a.kf[px];
    if (!surfel_ok(a.kg, s1)) return;
    const Rt32 T = load_pose_f32(a.pose);
    // T^-1 applied as R^T (x - t)
    const int i = px / a.kg.cols, j = px - i * a.kg.cols;
    const float3 uk = ray(a.kg, i, j);
    const float3 x1 = make_float3(s1.w * uk.x, s1.w * uk.y, s1.w * uk.z);
    const float3 d0 = make_float3(x1.x - T.t[0], x1.y - T.t[1], x1.z - T.t[2]);
    const float3 xs = make_float3(T.r[0] * d0.x + T.r[3] * d0.y + T.r[6] * d0.z,
                                  T.r[1] * d0.x + T.r[4] * d0.y + T.r[7] * d0.z,
                                  T.r[2] * d0.x + T.r[5] * d0.y + T.r[8] * d0.z);
    int si, sj;
    if (!project(a.sg, xs, si, sj)) return;
    const float4 s2 = a.scan[si * a.sg.cols + sj];
    if (!surfel_ok(a.sg, s2)) return;
    const float3 us = ray(a.sg, si, sj);
    const float3 q = transform(T, make_float3(s2.w * us.x, s2.w * us.y, s2.w * us.z));
    const float3 m = rotate(T, xyz(s2));
    const float3 n1 = xyz(s1);
    const float3 d = sub3(q, x1);
    if (!(dot3(d, d) <= a.d_max2)) return;
    if (!(dot3(m, n1) >= a.cos_theta)) return;
    const float un = dot3(uk, n1);
    if (!(fabsf(un) >= a.min_cos_inc)) return;
    const float r_new = s1.w + dot3(d, n1) / un;
    const float cf = (float)c;
    const float r_avg = (cf * s1.w + r_new) / (cf + 1.f);
    if (!range_ok(a.kg, r_avg)) return;
    const float3 n = make_float3(cf * n1.x + m.x, cf * n1.y + m.y, cf * n1.z + m.z);
    const float nn = sqrtf(dot3(n, n));
    if (!(nn > 0.f)) return;
    const float inv = 1.f / nn;
    a.kf[px] = make_float4(n.x * inv, n.y * inv, n.z * inv, r_avg);
    a.count[px] = (uint16_t)(c + 1 < a.max_count ? c + 1 : a.max_count);
}

__device__ __forceinline__ void fuse_fill(const FuseArgs &a, int p) {
    const int npix = a.sg.rows * a.sg.cols;
    if (p >= npix) return;
    const float4 s2 = a.scan[p];
    if (!surfel_ok(a.sg, s2)) return;
    const Rt32 T = load_pose_f32(a.pose);
    const int i = p / a.sg.cols, j = p - i * a.sg.cols;
    const float3 u = ray(a.sg, i, j);
    const float3 q = transform(T, make_float3(s2.w * u.x, s2.w * u.y, s2.w * u.z));
    const float rq = sqrtf(dot3(q, q));
    if (!range_ok(a.kg, rq)) return;
    int ki, kj;
    if (!project(a.kg, q, ki, kj)) return;
    const int kp = ki * a.kg.cols + kj;
    if (a.count[kp] != 0) return;
    const unsigned long long key = ((unsigned long long)__float_as_uint(rq) << 32) | (unsigned)p;
    atomicMin(&a.key[kp], key);
}

__global__ __launch_bounds__(kBlock) void k_fuse_update_fill(FuseArgs a, int update_blocks) {
    if ((int)blockIdx.x < update_blocks) fuse_update(a, blockIdx.x * kBlock + threadIdx.x);
    else fuse_fill(a, (blockIdx.x - update_blocks) * kBlock + threadIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_fuse_resolve(FuseArgs a) {
    const int npix = a.kg.rows * a.kg.cols;
    const int px = blockIdx.x * kBlock + threadIdx.x;
    if (px >= npix) return;
    if (a.count[px] != 0) return;
    const unsigned long long key = a.key[px];
    if (key == kNoKey) return;
    a.key[px] = kNoKey;
    const int p = (int)(key & 0xffffffffu);
    const float rq = __uint_as_float((unsigned)(key >> 32));
    const Rt32 T = load_pose_f32(a.pose);
    const float3 m = rotate(T, xyz(a.scan[p]));
    a.kf[px] = make_float4(m.x, m.y, m.z, rq);
    a.count[px] = 1;
}

ups_status launch_fuse(ups_context *ctx, const DGeom &sg, const float4 *scan, const DGeom &kg, float4 *kf,
                       uint16_t *count, const ups_pose *T, const ups_fuse_params &p, hipStream_t s) {
    FuseArgs a;
    a.sg = sg;
    a.kg = kg;
    a.scan = scan;
    a.kf = kf;
    a.count = count;
    a.key = ctx->fill_key;
    a.pose = T;
    a.d_max2 = p.d_max * p.d_max;
    a.cos_theta = p.cos_theta_max;
    a.min_cos_inc = p.min_cos_incidence;
    a.max_count = p.max_count;
    const int nk = kg.rows * kg.cols, ns = sg.rows * sg.cols;
    const int ub = (nk + kBlock - 1) / kBlock, fb = (ns + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_fuse_update_fill, dim3(ub + fb), dim3(kBlock), 0, s, a, ub);
    UPS_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_fuse_resolve, dim3((nk + kBlock - 1) / kBlock), dim3(kBlock), 0, s, a);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
