// Host-side internals of the library: the context (all device scratch memory,
// allocated once), error reporting, geometry validation and the per-geometry
// ray-table cache, plus the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ups_device.hpp"
#include "upslam.h"

namespace ups {

void set_error(const std::string &msg);

#define UPS_CHECK_HIP(expr)                                                                   \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess) {                                                               \
            ::ups::set_error(std::string(#expr) + ": " + hipGetErrorString(_e));              \
            return UPS_ERR_HIP;                                                               \
        }                                                                                     \
    } while (0)

#define UPS_REQUIRE(cond, msg)                                                                \
    do {                                                                                      \
        if (!(cond)) {                                                                        \
            ::ups::set_error(msg);                                                            \
            return UPS_ERR_INVALID_ARG;                                                       \
        }                                                                                     \
    } while (0)

struct LutEntry {
    int rows, cols;
    double el_top, d_el;
    float2 *row, *col;  // device
};

struct RegState;

}  // namespace ups

struct ups_context {
    int device = 0;
    int64_t max_pixels = 0;
    int32_t max_batch = 0;
    int64_t max_batch_pixels = 0;
    // scratch
    float4 *tmp_surfel = nullptr;  // a-trous ping-pong, max_pixels
    unsigned long long *fill_key = nullptr;  // fuse fill pass, max_pixels
    double *partials = nullptr;              // [2][kPartialStride][max_partial_blocks] block partials
    int64_t max_partial_blocks = 0;
    ups::RegState *state = nullptr;          // [2] registration state slots, then two counters (kSingleStateBytes)
    // ray tables
    float2 *lut_arena = nullptr;
    size_t lut_capacity = 0, lut_used = 0;  // in float2
    std::vector<ups::LutEntry> luts;
    std::vector<std::pair<int64_t, int>> tuned;  // autotuned pixels per thread by panorama size
    std::mutex mu;
};

namespace ups {

constexpr int kPartialStride = 32;  // doubles per block partial

// Block partials are stored by value: value v of block b at
// partials[v * pstride + b], pstride = the block capacity rounded up to a
// multiple of 16 (even, so that two consecutive blocks load as 16 bytes).
inline int64_t partial_stride(int64_t blocks) { return (blocks + 15) / 16 * 16; }

// Makes `dev` the current device for the scope and restores the caller's.
struct DeviceGuard {
    int prev = -1;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev) {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Validate a geometry and return its device view at pyramid level `level`
// (ray tables are uploaded on first use of the geometry).
ups_status device_geom(ups_context *ctx, const ups_geom *g, int level, hipStream_t stream, DGeom *out);
// The device view of a validated geometry at `level` over given level-0 ray
// tables (lut_row[rows], lut_col[cols]: (cos, sin) of elevations / azimuths).
DGeom geom_view(const ups_geom *g, int level, const float2 *lut_row, const float2 *lut_col);
ups_status check_ptr(const void *p, size_t align, const char *what);
ups_status check_geom(const ups_geom *g, const char *what);
ups_status check_icp_params(const ups_icp_params *p);
// rows and cols of g divisible by 2^(levels-1), cols by 64 * 2^(levels-1)
ups_status check_levels(const ups_geom *g, int levels, const char *what);
// Autotuned pixels per thread for batch launches over panoramas of about npix
// pixels (0 when ups_autotune has not run).
int autotuned_k(ups_context *ctx, int64_t npix);

// One panorama of a batched normals launch.
struct NormImg {
    DGeom g;
    const float *depth;
    float4 *out;     // surfel image
    float4 *tmp;     // a-trous ping-pong buffer of the same size
    float4 *pyr[3];  // its pyramid levels 1-3 (null past the batch's levels)
};

// Tiles of a panorama in the batched a-trous launches (at most 2^kNormTileBits:
// 64-pixel-wide tiles of 16 rows, cols <= 8192, rows <= 1024).
int normal_tiles(const DGeom &g);
constexpr int kNormTileBits = 13;
// tile_of[b]: (image << kNormTileBits) | tile of the image, for every block b.
// write_pyr: the last pass also writes every image's pyramid levels (pyr).
ups_status launch_normals_batch(const NormImg *imgs, const unsigned *tile_of, int total_tiles,
                                const ups_normal_params &p, int write_pyr, hipStream_t s);

// launchers (each returns UPS_OK or sets the error)
ups_status launch_normals(ups_context *ctx, const DGeom &g, const float *depth, float4 *surfel,
                          const ups_normal_params &p, hipStream_t s);
ups_status launch_subsample(const DGeom &g0, const float4 *src, int level, float4 *dst, hipStream_t s);
ups_status launch_correspondences(const DGeom &sg, const float4 *scan, const DGeom &kg, const float4 *kf,
                                  const ups_pose *T, float d_max, float cos_theta, int32_t *idx, uint8_t *inl,
                                  hipStream_t s);
ups_status launch_project_points(const DGeom &g, const float *xyz, int64_t n, int32_t *ii, int32_t *jj,
                                 hipStream_t s);
ups_status launch_fuse(ups_context *ctx, const DGeom &sg, const float4 *scan, const DGeom &kg, float4 *kf,
                       uint16_t *count, const ups_pose *T, const ups_fuse_params &p, hipStream_t s);

}  // namespace ups
