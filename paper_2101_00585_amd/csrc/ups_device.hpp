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
    int lshift;           // level (log2 of stride)
    float el_top, inv_d_el, az_scale;  // az_scale = cols / (2 pi)
    float r_min, r_max;
    int narrow;             // every row (with half a row of margin) lies within +-45 deg elevation
    const float2 *lut_row;  // [rows0] (cos el, sin el)
    const float2 *lut_col;  // [cols0] (cos az, sin az)
};

// Loads through explicit address spaces.  Pointers that reach a kernel inside
// a descriptor in memory are generic to the compiler, which would emit flat
// loads (counted on both the vector-memory and the LDS counters); these
// helpers issue global loads, and scalar loads for wave-uniform read-only
// tables.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
#define UPS_AS_GLOBAL __attribute__((address_space(1)))
#define UPS_AS_CONST __attribute__((address_space(4)))

__device__ __forceinline__ float4 ldg(const float4 *p, int idx) {
    const v4f v = ((const UPS_AS_GLOBAL v4f *)p)[idx];
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ldg(const float2 *p, int idx) {
    const v2f v = ((const UPS_AS_GLOBAL v2f *)p)[idx];
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ float ldg(const float *p, int idx) { return ((const UPS_AS_GLOBAL float *)p)[idx]; }
// The same with a non-negative index whose byte offset fits in 32 bits: the
// load takes the (wave-uniform) base in scalar registers and a 32-bit vector
// offset, with no 64-bit address arithmetic per lane.
__device__ __forceinline__ float4 ldg_u(const float4 *p, uint32_t idx) {
    const v4f v = *(const UPS_AS_GLOBAL v4f *)((const UPS_AS_GLOBAL char *)p + (idx << 4));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ldg_u(const float2 *p, uint32_t idx) {
    const v2f v = *(const UPS_AS_GLOBAL v2f *)((const UPS_AS_GLOBAL char *)p + (idx << 3));
    return make_float2(v.x, v.y);
}
// idx must be the same in every lane of the wavefront
__device__ __forceinline__ float2 lds_uniform(const float2 *p, int idx) {
    const v2f v = ((const UPS_AS_CONST v2f *)p)[idx];
    return make_float2(v.x, v.y);
}

// Validity tests combine their comparisons with non-short-circuit operators:
// no branches, so that loads feeding them are not moved into conditional code.
__device__ __forceinline__ bool range_ok(const DGeom &g, float r) { return (r > g.r_min) & (r <= g.r_max); }

__device__ __forceinline__ bool normal_ok(float4 s) { return (s.x != 0.f) | (s.y != 0.f) | (s.z != 0.f); }

__device__ __forceinline__ bool surfel_ok(const DGeom &g, float4 s) { return range_ok(g, s.w) & normal_ok(s); }

__device__ __forceinline__ float3 ray(const DGeom &g, int i, int j) {
    const float2 e = ldg(g.lut_row, i * g.stride);
    const float2 a = ldg(g.lut_col, j * g.stride);
    return make_float3(e.x * a.x, e.x * a.y, e.y);
}

// Ray of pixel (i, j) when i is the same in every lane (scalar row-table load).
__device__ __forceinline__ float3 ray_urow(const DGeom &g, int i, int j) {
    const float2 e = lds_uniform(g.lut_row, i * g.stride);
    const float2 a = ldg(g.lut_col, j * g.stride);
    return make_float3(e.x * a.x, e.x * a.y, e.y);
}

// atan(a) for |a| <= 1 in FP32 from a minimax polynomial a P(a^2) with the 8
// coefficients below (fitted for this library by linear programming on the
// maximum absolute error over [0, 1]: 2.9e-8 rad in exact arithmetic,
// 1.4e-7 rad when evaluated in FP32).
__device__ __forceinline__ float atan_unit(float a) {
    const float s = a * a;
    float p = -0.004214501939713955f;
    p = p * s + 0.022454990074038506f;
    p = p * s - 0.0567864254117012f;
    p = p * s + 0.09707822650671005f;
    p = p * s - 0.13935041427612305f;
    p = p * s + 0.19952043890953064f;
    p = p * s - 0.33330363035202026f;
    p = p * s + 0.999999463558197f;
    return a * p;
}

// atan2 from atan_unit and the octant symmetries atan(a) = pi/2 - atan(1/a),
// pi - ..., and the sign of y.  Undefined for x = y = 0 (callers exclude it).
__device__ __forceinline__ float atan2_fast(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const bool steep = ay > ax;
    const float mx = steep ? ay : ax, mn = steep ? ax : ay;
    float r = atan_unit(mn * __builtin_amdgcn_rcpf(mx));
    if (steep) r = 1.57079632679489662f - r;
    if (x < 0.f) r = 3.14159265358979324f - r;
    return copysignf(r, y);
}

// Nearest pixel centre of the direction of q: i = floor(fi + 1/2),
// j = floor(fj + 1/2) mod cols with fi = (el_top - el)/d_el and
// fj = az cols / (2 pi), az in [0, 2 pi).  False for the origin and rows
// outside [0, rows).  Branch-free: pi and pj are computed (and meaningless)
// whenever the result is false, so that callers can issue their loads
// unconditionally.
__device__ __forceinline__ bool project(const DGeom &g, float3 q, int &pi, int &pj) {
    const float rho = __builtin_amdgcn_sqrtf(q.x * q.x + q.y * q.y);
    bool ok;
    float el;
    if (g.narrow) {
        // the panorama lies within +-45 deg: steeper directions have no pixel
        // (this also excludes the origin)
        ok = fabsf(q.z) < rho;
        el = atan_unit(q.z * __builtin_amdgcn_rcpf(rho));
    } else {
        ok = (rho != 0.f) | (q.z != 0.f);
        el = atan2_fast(q.z, rho);
    }
    float az = atan2_fast(q.y, q.x);
    az = az < 0.f ? az + kTwoPi : az;
    const float fi = floorf((g.el_top - el) * g.inv_d_el + 0.5f);
    ok = ok & (fi >= 0.f) & (fi < (float)g.rows);
    int j = (int)floorf(az * g.az_scale + 0.5f);
    j = j >= g.cols ? j - g.cols : j;
    pi = (int)fi;
    pj = j;
    return ok;
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

// The association split in two phases so that a caller can overlap the
// keyframe gathers of one pixel with the scan loads of the next:
//   scan_side: transform the scan point and normal, project into the keyframe
//              and issue the keyframe loads (surfel and ray tables);
//   kf_side:   the Omega filter and the residual once those loads arrived.
struct Gather {
    float3 q, m;  // transformed point and normal
    int kf_index; // -1: no scan surfel or no keyframe pixel
    float4 s1;    // keyframe surfel
    float2 e, a;  // keyframe ray tables (cos, sin) of the row and the column
};

// Branch-free: every lane issues its three loads (lanes without a pixel read
// pixel 0) and carries kf_index = -1.
// kshift: 0 when kf is the level's own image; l when it is the level-0 image
// read at every 2^l-th row and column (pixel (i, j) of level l at
// (i cols_0 + j) 2^l with cols_0 = cols 2^l).
__device__ __forceinline__ Gather scan_side(const DGeom &sg, float4 s2, float2 e, float2 ca, const DGeom &kg,
                                            const float4 *__restrict__ kf, const Rt32 &T, int kshift = 0) {
    Gather G;
    const bool sok = surfel_ok(sg, s2);
    const float3 u = make_float3(e.x * ca.x, e.x * ca.y, e.y);
    const float3 p = make_float3(s2.w * u.x, s2.w * u.y, s2.w * u.z);
    G.q = transform(T, p);
    G.m = rotate(T, make_float3(s2.x, s2.y, s2.z));
    int ki, kj;
    const bool ok = project(kg, G.q, ki, kj) & sok;
    ki = ok ? ki : 0;
    kj = ok ? kj : 0;
    const uint32_t idx = (__umul24((uint32_t)ki, (uint32_t)kg.cols << kshift) + (uint32_t)kj) << kshift;
    G.kf_index = ok ? (int)idx : -1;
    G.s1 = ldg_u(kf, idx);
    G.e = ldg_u(kg.lut_row, (uint32_t)ki << kg.lshift);
    G.a = ldg_u(kg.lut_col, (uint32_t)kj << kg.lshift);
    return G;
}

__device__ __forceinline__ void kf_side(const DGeom &kg, const Gather &G, float d_max2, float cos_theta_max,
                                        bool &inlier, float &r, float3 &n1) {
    // branch-free up to the inlier decision: the gathered values are used on
    // every path, so their loads stay where scan_side issued them
    float3 d;
    {
        // no FMA contraction: q - s1 must vanish exactly when the pose is the
        // identity and q, s1 are the same pixel's point
#pragma clang fp contract(off)
        const float3 uk = make_float3(G.e.x * G.a.x, G.e.x * G.a.y, G.e.y);
        const float3 x1 = make_float3(G.s1.w * uk.x, G.s1.w * uk.y, G.s1.w * uk.z);
        d = sub3(G.q, x1);
    }
    n1 = make_float3(G.s1.x, G.s1.y, G.s1.z);
    r = dot3(d, n1);
    inlier = (G.kf_index >= 0) & surfel_ok(kg, G.s1) & (dot3(d, d) <= d_max2) & (dot3(G.m, n1) >= cos_theta_max);
}

// ---- world-frame variant (precision study): points carried in world
// coordinates in FP32.  T is the scan's world pose, W the keyframe's; the
// scan point q = T p is re-expressed in the keyframe frame, W^T (q - W.t), only
// to find its pixel; the keyframe surfel is taken to the world, s1 = W x1,
// n1 = W.R n1, and the residual and Jacobian are formed from world
// coordinates.  At kilometre offsets every world coordinate carries the FP32
// rounding of its magnitude.
__device__ __forceinline__ float3 inv_transform(const Rt32 &T, float3 y) {
    const float3 d = make_float3(y.x - T.t[0], y.y - T.t[1], y.z - T.t[2]);
    return make_float3(T.r[0] * d.x + T.r[3] * d.y + T.r[6] * d.z, T.r[1] * d.x + T.r[4] * d.y + T.r[7] * d.z,
                       T.r[2] * d.x + T.r[5] * d.y + T.r[8] * d.z);
}

__device__ __forceinline__ Gather scan_side_world(const DGeom &sg, float4 s2, float2 e, float2 ca, const DGeom &kg,
                                                  const float4 *__restrict__ kf, const Rt32 &T, const Rt32 &W,
                                                  int kshift = 0) {
    Gather G;
    G.kf_index = -1;
    if (!surfel_ok(sg, s2)) return G;
    const float3 u = make_float3(e.x * ca.x, e.x * ca.y, e.y);
    const float3 p = make_float3(s2.w * u.x, s2.w * u.y, s2.w * u.z);
    G.q = transform(T, p);
    G.m = rotate(T, make_float3(s2.x, s2.y, s2.z));
    int ki, kj;
    if (!project(kg, inv_transform(W, G.q), ki, kj)) return G;
    G.kf_index = (ki * (kg.cols << kshift) + kj) << kshift;
    G.s1 = ldg(kf, G.kf_index);
    G.e = ldg(kg.lut_row, ki * kg.stride);
    G.a = ldg(kg.lut_col, kj * kg.stride);
    return G;
}

__device__ __forceinline__ void kf_side_world(const DGeom &kg, const Gather &G, const Rt32 &W, float d_max2,
                                              float cos_theta_max, bool &inlier, float &r, float3 &n1) {
    inlier = false;
    r = 0.f;
    n1 = make_float3(0.f, 0.f, 0.f);
    if (G.kf_index < 0 || !surfel_ok(kg, G.s1)) return;
    const float3 uk = make_float3(G.e.x * G.a.x, G.e.x * G.a.y, G.e.y);
    const float3 s1 = transform(W, make_float3(G.s1.w * uk.x, G.s1.w * uk.y, G.s1.w * uk.z));
    n1 = rotate(W, make_float3(G.s1.x, G.s1.y, G.s1.z));
    const float3 d = sub3(G.q, s1);
    if (!(dot3(d, d) <= d_max2)) return;
    if (!(dot3(G.m, n1) >= cos_theta_max)) return;
    inlier = true;
    r = dot3(d, n1);
}

// One projective correspondence of Equation 1 (Section III-B).
struct Pair {
    int kf_index;  // -1 when the scan pixel has no surfel or projects outside
    bool inlier;   // passes Omega_{d,theta}
    float r;       // (q - s1).n1
    float3 q, n1;  // J = [q x n1, n1]
};

template <bool UNIFORM_ROW = false>
__device__ __forceinline__ Pair associate(const DGeom &sg, float4 s2, int i, int j, const DGeom &kg,
                                          const float4 *__restrict__ kf, const Rt32 &T, float d_max2,
                                          float cos_theta_max) {
    Pair pr;
    pr.kf_index = -1;
    pr.inlier = false;
    pr.r = 0.f;
    if (!surfel_ok(sg, s2)) return pr;
    float3 u = UNIFORM_ROW ? ray_urow(sg, i, j) : ray(sg, i, j);
    float3 p = make_float3(s2.w * u.x, s2.w * u.y, s2.w * u.z);
    float3 q = transform(T, p);
    float3 m = rotate(T, xyz(s2));
    int ki, kj;
    if (!project(kg, q, ki, kj)) return pr;
    pr.kf_index = ki * kg.cols + kj;
    float4 s1 = ldg(kf, pr.kf_index);
    if (!surfel_ok(kg, s1)) return pr;
    float3 uk = ray(kg, ki, kj);
    float3 d;
    {
        // no FMA contraction: q - s1 must vanish exactly when the pose is the
        // identity and q, s1 are the same pixel's point
#pragma clang fp contract(off)
        const float3 x1 = make_float3(s1.w * uk.x, s1.w * uk.y, s1.w * uk.z);
        d = sub3(q, x1);
    }
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
