// Panorama formation (UPSLAM Section III-A) on gfx950: the measurements of
// one sweep, each in the frame of its firing instant, are moved into the
// frame of a single instant and projected into a panoramic image that keeps
// the nearest return per pixel.
//
//   k_splat_sweep    one thread per measurement: point, per-column transform
//                    (read once per column from a table in memory), projection,
//                    and a 64-bit atomicMin on (FP32 bits of the range, index)
//                    into the pixel's key: the nearest return wins, the
//                    smaller measurement index among equal ranges;
//   k_splat_resolve  one thread per output pixel: the winner's range (0 where
//                    nothing landed), and the key reset to all-ones.
// The keys are the context's fill scratch, all-ones between calls.
#include "ups_internal.hpp"

namespace ups {

namespace {

constexpr unsigned long long kEmpty = ~0ull;
constexpr int kSplatBlock = 256;

__global__ __launch_bounds__(kSplatBlock) void k_splat_sweep(DGeom rg, const float *__restrict__ raw,
                                                             const float *__restrict__ col_T, DGeom og,
                                                             unsigned long long *__restrict__ key) {
    const int n = rg.rows * rg.cols;
    const int px = blockIdx.x * kSplatBlock + threadIdx.x;
    if (px >= n) return;
    const float r = raw[px];
    if (!range_ok(rg, r)) return;
    const int i = px / rg.cols, j = px - i * rg.cols;
    const float3 u = ray(rg, i, j);
    float3 y = make_float3(r * u.x, r * u.y, r * u.z);
    if (col_T) {
        const float *C = col_T + 12 * (size_t)j;
        Rt32 T;
#pragma unroll
        for (int k = 0; k < 9; k++) T.r[k] = C[k];
#pragma unroll
        for (int k = 0; k < 3; k++) T.t[k] = C[9 + k];
        y = transform(T, y);
    }
    const float ry = __builtin_amdgcn_sqrtf(y.x * y.x + y.y * y.y + y.z * y.z);
    if (!range_ok(og, ry)) return;
    int oi, oj;
    if (!project(og, y, oi, oj)) return;
    const unsigned long long k = ((unsigned long long)__float_as_uint(ry) << 32) | (unsigned int)px;
    atomicMin(&key[(size_t)oi * og.cols + oj], k);
}

__global__ __launch_bounds__(kSplatBlock) void k_splat_resolve(int n, unsigned long long *__restrict__ key,
                                                               float *__restrict__ out) {
    const int q = blockIdx.x * kSplatBlock + threadIdx.x;
    if (q >= n) return;
    const unsigned long long k = key[q];
    out[q] = k == kEmpty ? 0.f : __uint_as_float((unsigned int)(k >> 32));
    if (k != kEmpty) key[q] = kEmpty;
}

}  // namespace

}  // namespace ups

using namespace ups;

extern "C" ups_status ups_splat_sweep(ups_context *ctx, const ups_geom *raw_g, const float *raw_range_d,
                                      const float *col_T_d, const ups_geom *out_g, float *depth_d, void *stream) {
    UPS_REQUIRE(ctx, "context is null");
    ups_status st;
    if ((st = check_ptr(raw_range_d, 4, "raw ranges")) != UPS_OK) return st;
    if ((st = check_ptr(depth_d, 4, "depth")) != UPS_OK) return st;
    if (col_T_d && (st = check_ptr(col_T_d, 4, "column transforms")) != UPS_OK) return st;
    UPS_REQUIRE((const void *)raw_range_d != (const void *)depth_d, "raw ranges and depth must not alias");
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    hipStream_t s = (hipStream_t)stream;
    DGeom rg, og;
    if ((st = device_geom(ctx, raw_g, 0, s, &rg)) != UPS_OK) return st;
    if ((st = device_geom(ctx, out_g, 0, s, &og)) != UPS_OK) return st;
    const int64_t nout = (int64_t)out_g->rows * out_g->cols;
    if (nout > ctx->max_pixels) {
        set_error("output panorama larger than the context's max_pixels");
        return UPS_ERR_WORKSPACE;
    }
    const int nraw = raw_g->rows * raw_g->cols;
    hipLaunchKernelGGL(k_splat_sweep, dim3((nraw + kSplatBlock - 1) / kSplatBlock), dim3(kSplatBlock), 0, s, rg,
                       raw_range_d, col_T_d, og, ctx->fill_key);
    UPS_CHECK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_splat_resolve, dim3((int)((nout + kSplatBlock - 1) / kSplatBlock)), dim3(kSplatBlock), 0, s,
                       (int)nout, ctx->fill_key, depth_d);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}
