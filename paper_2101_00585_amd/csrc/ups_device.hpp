// Device-side building blocks shared by the registration, fusion and normal
// kernels: panorama geometry with FP32 ray tables, spherical projection,
// rigid transforms in FP32 and the per-pixel association of Section III-B.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "upslam.h"

namespace ups {

constexpr float kTwoPi = 6.28318530717958647692f;
constexpr int kBlock = 256;  // threads per workgroup for the per-pixel kernels

// Panorama geometry of one pyramid level as the kernels see it.  Ray tables
// hold (cos, sin) of every level-0 row elevation and column azimuth, computed
// in FP64 and rounded to FP32; level l reads every 2^l-th entry.
struct DGeom {
    int rows, cols;       // at this level
    int stride;           // 2^level into the level-0 ray tables
    float el_top, inv_d_el, az_scale;  // az_scale = cols / (2 pi)
    float r_min, r_max;
    const float2 *lut_row;  // [rows0] (cos el, sin el)
    const float2 *lut_col;  // [cols0] (cos az, sin az)
};

__device__ __forceinline__ bool range_ok(const DGeom &g, float r) { return r > g.r_min && r <= g.r_max; }

__device__ __forceinline__ bool normal_ok(float4 s) { return s.x != 0.f || s.y != 0.f || s.z != 0.f; }

__device__ __forceinline__ bool surfel_ok(const DGeom &g, float4 s) { return range_ok(g, s.w) && normal_ok(s); }

__device__ __forceinline__ float3 ray(const DGeom &g, int i, int j) {
    float2 e = g.lut_row[i * g.stride];
    float2 a = g.lut_col[j * g.stride];
    return make_float3(e.x * a.x, e.x * a.y, e.y);
}

// Nearest pixel centre of the direction of q: i = floor(fi + 1/2),
// j = floor(fj + 1/2) mod cols with fi = (el_top - el)/d_el and
// fj = az cols / (2 pi), az in [0, 2 pi).  False for the origin and rows
// outside [0, rows).
__device__ __forceinline__ bool project(const DGeom &g, float3 q, int &pi, int &pj) {
    float rho = sqrtf(q.x * q.x + q.y * q.y);
    if (rho == 0.f && q.z == 0.f) return false;
    float el = atan2f(q.z, rho);
    float az = atan2f(q.y, q.x);
    if (az < 0.f) az += kTwoPi;
    float fi = floorf((g.el_top - el) * g.inv_d_el + 0.5f);
    if (!(fi >= 0.f && fi < (float)g.rows)) return false;
    int j = (int)floorf(az * g.az_scale + 0.5f);
    if (j >= g.cols) j -= g.cols;
    pi = (int)fi;
    pj = j;
    return true;
}

struct Rt32 {
    float r[9];
    float t[3];
};

__device__ __forceinline__ Rt32 load_pose_f32(const ups_pose *T) {
    Rt32 o;
#pragma unroll
    for (int k = 0; k < 9; k++) o.r[k] = (float)T->R[k];
#pragma unroll
    for (int k = 0; k < 3; k++) o.t[k] = (float)T->t[k];
    return o;
}

__device__ __forceinline__ float3 rotate(const Rt32 &T, float3 x) {
    return make_float3(T.r[0] * x.x + T.r[1] * x.y + T.r[2] * x.z, T.r[3] * x.x + T.r[4] * x.y + T.r[5] * x.z,
                       T.r[6] * x.x + T.r[7] * x.y + T.r[8] * x.z);
}

__device__ __forceinline__ float3 transform(const Rt32 &T, float3 x) {
    float3 y = rotate(T, x);
    return make_float3(y.x + T.t[0], y.y + T.t[1], y.z + T.t[2]);
}

__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

__device__ __forceinline__ float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }

__device__ __forceinline__ float3 xyz(float4 s) { return make_float3(s.x, s.y, s.z); }

// One projective correspondence of Equation 1 (Section III-B).
struct Pair {
    int kf_index;  // -1 when the scan pixel has no surfel or projects outside
    bool inlier;   // passes Omega_{d,theta}
    float r;       // (q - s1).n1
    float3 q, n1;  // J = [q x n1, n1]
};

__device__ __forceinline__ Pair associate(const DGeom &sg, float4 s2, int i, int j, const DGeom &kg,
                                          const float4 *__restrict__ kf, const Rt32 &T, float d_max2,
                                          float cos_theta_max) {
    // no FMA contraction here: q - s1 must vanish exactly when the pose is the
    // identity and q, s1 are the same pixel's point
#pragma clang fp contract(off)
    Pair pr;
    pr.kf_index = -1;
    pr.inlier = false;
    pr.r = 0.f;
    if (!surfel_ok(sg, s2)) return pr;
    float3 u = ray(sg, i, j);
    float3 p = make_float3(s2.w * u.x, s2.w * u.y, s2.w * u.z);
    float3 q = transform(T, p);
    float3 m = rotate(T, xyz(s2));
    int ki, kj;
    if (!project(kg, q, ki, kj)) return pr;
    pr.kf_index = ki * kg.cols + kj;
    float4 s1 = kf[pr.kf_index];
    if (!surfel_ok(kg, s1)) return pr;
    float3 uk = ray(kg, ki, kj);
    float3 x1 = make_float3(s1.w * uk.x, s1.w * uk.y, s1.w * uk.z);
    float3 d = sub3(q, x1);
    float3 n1 = xyz(s1);
    if (!(dot3(d, d) <= d_max2)) return pr;
    if (!(dot3(m, n1) >= cos_theta_max)) return pr;
    pr.inlier = true;
    pr.r = dot3(d, n1);
    pr.q = q;
    pr.n1 = n1;
    return pr;
}

}  // namespace ups
