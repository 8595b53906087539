// C ABI entry points (include/upslam.h): argument validation, the context
// with all device scratch memory, the per-geometry ray tables, and dispatch to
// the kernel launchers.
#include <atomic>
#include <cmath>
#include <string>

#include "ups_icp.hpp"

namespace ups {

static thread_local std::string g_last_error;
static std::atomic<int> g_reverse_tiles{0};
static std::atomic<unsigned> g_level_spin_limit{ups::kLevelSpinLimit};

void set_error(const std::string &msg) { g_last_error = msg; }

ups_status check_ptr(const void *p, size_t align, const char *what) {
    if (!p) {
        set_error(std::string(what) + " is null");
        return UPS_ERR_INVALID_ARG;
    }
    if (((uintptr_t)p) % align != 0) {
        set_error(std::string(what) + " is not " + std::to_string(align) + "-byte aligned");
        return UPS_ERR_INVALID_ARG;
    }
    return UPS_OK;
}


ups_status check_geom(const ups_geom *g, const char *what) {
    UPS_REQUIRE(g != nullptr, std::string(what) + " geometry is null");
    UPS_REQUIRE(g->rows >= 2 && g->rows <= 4096, std::string(what) + ": rows must be in [2, 4096]");
    UPS_REQUIRE(g->cols >= 64 && g->cols <= 16384 && g->cols % 64 == 0,
                std::string(what) + ": cols must be a multiple of 64 in [64, 16384]");
    UPS_REQUIRE(std::isfinite(g->el_top) && std::isfinite(g->d_el) && g->d_el > 0.0,
                std::string(what) + ": el_top / d_el must be finite with d_el > 0");
    UPS_REQUIRE(std::isfinite(g->r_max) && g->r_min >= 0.0 && g->r_max > g->r_min,
                std::string(what) + ": need 0 <= r_min < r_max");
    return UPS_OK;
}

ups_status device_geom(ups_context *ctx, const ups_geom *g, int level, hipStream_t stream, DGeom *out) {
    ups_status st = check_geom(g, "panorama");
    if (st != UPS_OK) return st;
    LutEntry *e = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto &x : ctx->luts)
            if (x.rows == g->rows && x.cols == g->cols && x.el_top == g->el_top && x.d_el == g->d_el) e = &x;
        if (!e) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (stream) (void)hipStreamIsCapturing(stream, &cs);
            UPS_REQUIRE(cs == hipStreamCaptureStatusNone,
                        "first use of a panorama geometry during stream capture: call once before capturing");
            const size_t need = (size_t)g->rows + g->cols;
            if (ctx->lut_used + need > ctx->lut_capacity) {
                set_error("ray-table arena full (too many distinct geometries)");
                return UPS_ERR_WORKSPACE;
            }
            std::vector<float2> h(need);
            // (cos, sin) of row elevations and column azimuths in FP64, rounded to FP32
            for (int i = 0; i < g->rows; i++) {
                const double el = g->el_top - (double)i * g->d_el;
                h[i] = make_float2((float)std::cos(el), (float)std::sin(el));
            }
            for (int j = 0; j < g->cols; j++) {
                const double az = 2.0 * M_PI * (double)j / (double)g->cols;
                h[g->rows + j] = make_float2((float)std::cos(az), (float)std::sin(az));
            }
            float2 *dst = ctx->lut_arena + ctx->lut_used;
            UPS_CHECK_HIP(hipMemcpy(dst, h.data(), need * sizeof(float2), hipMemcpyHostToDevice));
            ctx->lut_used += need;
            ctx->luts.push_back(LutEntry{g->rows, g->cols, g->el_top, g->d_el, dst, dst + g->rows});
            e = &ctx->luts.back();
        }
    }
    *out = geom_view(g, level, e->row, e->col);
    return UPS_OK;
}

DGeom geom_view(const ups_geom *g, int level, const float2 *lut_row, const float2 *lut_col) {
    const int s = 1 << level;
    DGeom d;
    d.rows = g->rows >> level;
    d.cols = g->cols >> level;
    d.stride = s;
    d.lshift = level;
    d.el_top = (float)g->el_top;
    d.inv_d_el = (float)(1.0 / (g->d_el * s));
    d.az_scale = (float)((double)d.cols / (2.0 * M_PI));
    d.r_min = (float)g->r_min;
    d.r_max = (float)g->r_max;
    {
        const double dl = g->d_el * s, half = 0.5 * dl;
        const double top = g->el_top + half, bottom = g->el_top - (d.rows - 1) * dl - half;
        d.narrow = (top < M_PI / 4 - 1e-6 && bottom > -M_PI / 4 + 1e-6) ? 1 : 0;
    }
    d.lut_row = lut_row;
    d.lut_col = lut_col;
    return d;
}

ups_status check_icp_params(const ups_icp_params *p) {
    UPS_REQUIRE(p != nullptr, "icp params is null");
    UPS_REQUIRE(p->levels >= 1 && p->levels <= 4, "levels must be in [1, 4]");
    for (int l = 0; l < p->levels; l++) {
        UPS_REQUIRE(p->iters[l] >= 0 && p->iters[l] <= 1000, "iters must be in [0, 1000]");
        UPS_REQUIRE(p->d_max[l] > 0.f && std::isfinite(p->d_max[l]), "d_max must be > 0");
    }
    UPS_REQUIRE(p->cos_theta_max >= -1.f && p->cos_theta_max <= 1.f, "cos_theta_max must be in [-1, 1]");
    UPS_REQUIRE(p->stop_update_norm >= 0.0, "stop_update_norm must be >= 0");
    UPS_REQUIRE(p->precision >= UPS_PREC_KAHAN_F64 && p->precision <= UPS_PREC_F64, "unknown precision mode");
    UPS_REQUIRE(p->irls_delta == 0.f || (p->irls_delta >= 1e-6f && std::isfinite(p->irls_delta)),
                "irls_delta must be 0 or a finite value >= 1e-6");
    UPS_REQUIRE(p->irls_delta == 0.f || p->precision == UPS_PREC_KAHAN_F64,
                "the IRLS objective (irls_delta > 0) needs precision UPS_PREC_KAHAN_F64");
    return UPS_OK;
}

ups_status check_levels(const ups_geom *g, int levels, const char *what) {
    const int s = 1 << (levels - 1);
    UPS_REQUIRE(g->rows % s == 0 && g->rows / s >= 2,
                std::string(what) + ": rows must be divisible by 2^(levels-1)");
    UPS_REQUIRE(g->cols % (64 * s) == 0,
                std::string(what) + ": cols must be divisible by 64 * 2^(levels-1)");
    return UPS_OK;
}

}  // namespace ups

using namespace ups;

namespace ups {
bool debug_reverse_tiles() { return g_reverse_tiles.load(std::memory_order_relaxed) != 0; }
unsigned level_spin_limit() { return g_level_spin_limit.load(std::memory_order_relaxed); }
}  // namespace ups

extern "C" {

const char *ups_last_error(void) { return g_last_error.c_str(); }

ups_status ups_debug_reverse_tile_order(int32_t reversed) {
    g_reverse_tiles.store(reversed ? 1 : 0, std::memory_order_relaxed);
    return UPS_OK;
}

ups_status ups_debug_level_spin_limit(int64_t polls) {
    UPS_REQUIRE(polls < ((int64_t)1 << 32), "polls must be below 2^32");
    g_level_spin_limit.store(polls < 0 ? kLevelSpinLimit : (unsigned)polls, std::memory_order_relaxed);
    return UPS_OK;
}

ups_status ups_context_create(ups_context **out, int device, int64_t max_pixels, int32_t max_batch,
                              int64_t max_batch_pixels) {
    UPS_REQUIRE(out != nullptr, "out is null");
    *out = nullptr;
    UPS_REQUIRE(max_pixels >= 64 && max_pixels <= (int64_t)1 << 26, "max_pixels must be in [64, 2^26]");
    UPS_REQUIRE(max_batch >= 0 && max_batch <= 65536, "max_batch must be in [0, 65536]");
    UPS_REQUIRE(max_batch_pixels >= 0 && max_batch_pixels <= (int64_t)1 << 31, "max_batch_pixels out of range");
    int ndev = 0;
    UPS_CHECK_HIP(hipGetDeviceCount(&ndev));
    UPS_REQUIRE(device >= 0 && device < ndev, "no such device");
    DeviceGuard dg(device);
    UPS_CHECK_HIP(dg.err);
    ups_context *c = new ups_context();
    c->device = device;
    c->max_pixels = max_pixels;
    c->max_batch = max_batch;
    c->max_batch_pixels = max_batch_pixels;
    c->max_partial_blocks = partial_stride(max_pixels / kBlock + 64);  // single registrations (batches own theirs)
    c->lut_capacity = (size_t)1 << 20;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&c->tmp_surfel, max_pixels * sizeof(float4));
    if (e == hipSuccess) e = hipMalloc(&c->fill_key, max_pixels * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(c->fill_key, 0xFF, max_pixels * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&c->partials, 2 * c->max_partial_blocks * kPartialStride * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->state, kSingleStateBytes);
    if (e == hipSuccess) e = hipMemset(c->state, 0, kSingleStateBytes);
    if (e == hipSuccess) e = hipMalloc(&c->lut_arena, c->lut_capacity * sizeof(float2));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        set_error(std::string("context allocation failed: ") + hipGetErrorString(e));
        ups_context_destroy(c);
        return UPS_ERR_HIP;
    }
    *out = c;
    return UPS_OK;
}

void ups_context_destroy(ups_context *c) {
    if (!c) return;
    DeviceGuard dg(c->device);
    (void)hipFree(c->tmp_surfel);
    (void)hipFree(c->fill_key);
    (void)hipFree(c->partials);
    (void)hipFree(c->state);
    (void)hipFree(c->lut_arena);
    delete c;
}

ups_status ups_panorama_normals(ups_context *ctx, const ups_geom *g, const float *depth_d, float *surfel_d,
                                const ups_normal_params *p, void *stream) {
    UPS_REQUIRE(ctx && p, "context / params is null");
    ups_status st;
    if ((st = check_ptr(depth_d, 4, "depth")) != UPS_OK) return st;
    if ((st = check_ptr(surfel_d, 16, "surfel")) != UPS_OK) return st;
    UPS_REQUIRE((const void *)depth_d != (const void *)surfel_d, "surfel must not alias depth");
    UPS_REQUIRE(p->atrous_levels >= 0 && p->atrous_levels <= 3, "atrous_levels must be in [0, 3]");
    UPS_REQUIRE(p->sigma_n > 0.f && p->sigma_r > 0.f && p->max_rel_jump >= 0.f, "sigmas must be > 0");
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    DGeom dg0;
    if ((st = device_geom(ctx, g, 0, (hipStream_t)stream, &dg0)) != UPS_OK) return st;
    if ((int64_t)g->rows * g->cols > ctx->max_pixels) {
        set_error("panorama larger than the context's max_pixels");
        return UPS_ERR_WORKSPACE;
    }
    return launch_normals(ctx, dg0, depth_d, (float4 *)surfel_d, *p, (hipStream_t)stream);
}

ups_status ups_pyramid_level(ups_context *ctx, const ups_geom *g, const float *surfel_d, int32_t level,
                             float *out_d, void *stream) {
    UPS_REQUIRE(ctx, "context is null");
    ups_status st;
    if ((st = check_ptr(surfel_d, 16, "surfel")) != UPS_OK) return st;
    if ((st = check_ptr(out_d, 16, "out")) != UPS_OK) return st;
    UPS_REQUIRE(level >= 1 && level <= 3, "level must be in [1, 3]");
    if ((st = check_geom(g, "panorama")) != UPS_OK) return st;
    UPS_REQUIRE(g->rows % (1 << level) == 0 && g->cols % (1 << level) == 0, "rows/cols not divisible by 2^level");
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    DGeom d0;
    if ((st = device_geom(ctx, g, 0, (hipStream_t)stream, &d0)) != UPS_OK) return st;
    return launch_subsample(d0, (const float4 *)surfel_d, level, (float4 *)out_d, (hipStream_t)stream);
}

// world_kf: null for the keyframe-frame path, else the keyframe's world pose.
static ups_status register_impl(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                                const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *world_kf,
                                const ups_pose *init_d, const ups_icp_params *p, ups_icp_result *result_d,
                                void *stream) {
    UPS_REQUIRE(ctx, "context is null");
    ups_status st;
    if ((st = check_icp_params(p)) != UPS_OK) return st;
    if ((st = check_ptr(scan_surfel_d, 16, "scan surfel")) != UPS_OK) return st;
    if ((st = check_ptr(kf_surfel_d, 16, "keyframe surfel")) != UPS_OK) return st;
    if ((st = check_ptr(init_d, 8, "init pose")) != UPS_OK) return st;
    if ((st = check_ptr(result_d, 8, "result")) != UPS_OK) return st;
    if ((st = check_geom(scan_g, "scan")) != UPS_OK) return st;
    if ((st = check_geom(kf_g, "keyframe")) != UPS_OK) return st;
    if ((st = check_levels(scan_g, p->levels, "scan")) != UPS_OK) return st;
    if ((st = check_levels(kf_g, p->levels, "keyframe")) != UPS_OK) return st;
    if ((int64_t)scan_g->rows * scan_g->cols > ctx->max_pixels || (int64_t)kf_g->rows * kf_g->cols > ctx->max_pixels) {
        set_error("panorama larger than the context's max_pixels");
        return UPS_ERR_WORKSPACE;
    }
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    Inst I;
    memset(&I, 0, sizeof(I));
    for (int l = 0; l < p->levels; l++) {
        if ((st = device_geom(ctx, scan_g, l, (hipStream_t)stream, &I.sg[l])) != UPS_OK) return st;
        if ((st = device_geom(ctx, kf_g, l, (hipStream_t)stream, &I.kg[l])) != UPS_OK) return st;
        // every level is read from the level-0 images
        I.scan[l] = (const float4 *)scan_surfel_d;
        I.kf[l] = (const float4 *)kf_surfel_d;
    }
    I.state = ctx->state;
    I.xsync = xsync_of(ctx->state);
    I.partials = ctx->partials;
    I.pstride = (int)ctx->max_partial_blocks;
    I.res = result_d;
    if (world_kf) {
        I.world = 1;
        memcpy(I.wR, world_kf->R, sizeof(I.wR));
        memcpy(I.wt, world_kf->t, sizeof(I.wt));
    }
    return launch_register(I, init_d, *p, (hipStream_t)stream);
}

ups_status ups_register_scan(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                             const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *init_d,
                             const ups_icp_params *p, ups_icp_result *result_d, void *stream) {
    return register_impl(ctx, scan_g, scan_surfel_d, kf_g, kf_surfel_d, nullptr, init_d, p, result_d, stream);
}

static ups_status check_world_pose(const ups_pose *w) {
    UPS_REQUIRE(w, "world pose is null");
    for (double v : w->R) UPS_REQUIRE(std::isfinite(v), "world pose is not finite");
    for (double v : w->t) UPS_REQUIRE(std::isfinite(v), "world pose is not finite");
    return UPS_OK;
}

ups_status ups_register_scan_world(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                                   const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *world_kf_h,
                                   const ups_pose *init_d, const ups_icp_params *p, ups_icp_result *result_d,
                                   void *stream) {
    ups_status st;
    if ((st = check_world_pose(world_kf_h)) != UPS_OK) return st;
    UPS_REQUIRE(p == nullptr || p->irls_delta == 0.f, "the world-frame variant has no IRLS objective");
    return register_impl(ctx, scan_g, scan_surfel_d, kf_g, kf_surfel_d, world_kf_h, init_d, p, result_d, stream);
}

ups_status ups_fuse_scan(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                         const ups_geom *kf_g, float *kf_surfel_d, uint16_t *kf_count_d, const ups_pose *T_d,
                         const ups_fuse_params *p, void *stream) {
    UPS_REQUIRE(ctx && p, "context / params is null");
    ups_status st;
    if ((st = check_ptr(scan_surfel_d, 16, "scan surfel")) != UPS_OK) return st;
    if ((st = check_ptr(kf_surfel_d, 16, "keyframe surfel")) != UPS_OK) return st;
    if ((st = check_ptr(kf_count_d, 2, "keyframe count")) != UPS_OK) return st;
    if ((st = check_ptr(T_d, 8, "pose")) != UPS_OK) return st;
    UPS_REQUIRE(p->d_max > 0.f && p->max_count >= 1 && p->max_count <= 65535 && p->min_cos_incidence >= 0.f,
                "invalid fuse params");
    UPS_REQUIRE((const void *)scan_surfel_d != (const void *)kf_surfel_d, "scan and keyframe must not alias");
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    DGeom sg, kg;
    if ((st = device_geom(ctx, scan_g, 0, (hipStream_t)stream, &sg)) != UPS_OK) return st;
    if ((st = device_geom(ctx, kf_g, 0, (hipStream_t)stream, &kg)) != UPS_OK) return st;
    if ((int64_t)kf_g->rows * kf_g->cols > ctx->max_pixels) {
        set_error("keyframe larger than the context's max_pixels");
        return UPS_ERR_WORKSPACE;
    }
    return launch_fuse(ctx, sg, (const float4 *)scan_surfel_d, kg, (float4 *)kf_surfel_d, kf_count_d, T_d, *p,
                       (hipStream_t)stream);
}

static ups_status correspondences_impl(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                                       const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *world_kf,
                                       const ups_pose *T_d, float d_max, float cos_theta_max, int32_t *kf_index_d,
                                       uint8_t *inlier_d, void *stream) {
    UPS_REQUIRE(ctx, "context is null");
    ups_status st;
    if ((st = check_ptr(scan_surfel_d, 16, "scan surfel")) != UPS_OK) return st;
    if ((st = check_ptr(kf_surfel_d, 16, "keyframe surfel")) != UPS_OK) return st;
    if ((st = check_ptr(T_d, 8, "pose")) != UPS_OK) return st;
    if ((st = check_ptr(kf_index_d, 4, "kf_index")) != UPS_OK) return st;
    if ((st = check_ptr(inlier_d, 1, "inlier")) != UPS_OK) return st;
    UPS_REQUIRE(d_max > 0.f, "d_max must be > 0");
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    DGeom sg, kg;
    if ((st = device_geom(ctx, scan_g, 0, (hipStream_t)stream, &sg)) != UPS_OK) return st;
    if ((st = device_geom(ctx, kf_g, 0, (hipStream_t)stream, &kg)) != UPS_OK) return st;
    if (world_kf)
        return launch_correspondences_world(sg, (const float4 *)scan_surfel_d, kg, (const float4 *)kf_surfel_d, T_d,
                                            *world_kf, d_max, cos_theta_max, kf_index_d, inlier_d,
                                            (hipStream_t)stream);
    return launch_correspondences(sg, (const float4 *)scan_surfel_d, kg, (const float4 *)kf_surfel_d, T_d, d_max,
                                  cos_theta_max, kf_index_d, inlier_d, (hipStream_t)stream);
}

ups_status ups_correspondences(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                               const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *T_d, float d_max,
                               float cos_theta_max, int32_t *kf_index_d, uint8_t *inlier_d, void *stream) {
    return correspondences_impl(ctx, scan_g, scan_surfel_d, kf_g, kf_surfel_d, nullptr, T_d, d_max, cos_theta_max,
                                kf_index_d, inlier_d, stream);
}

ups_status ups_correspondences_world(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                                     const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *world_kf_h,
                                     const ups_pose *T_d, float d_max, float cos_theta_max, int32_t *kf_index_d,
                                     uint8_t *inlier_d, void *stream) {
    ups_status st;
    if ((st = check_world_pose(world_kf_h)) != UPS_OK) return st;
    return correspondences_impl(ctx, scan_g, scan_surfel_d, kf_g, kf_surfel_d, world_kf_h, T_d, d_max,
                                cos_theta_max, kf_index_d, inlier_d, stream);
}

ups_status ups_project_points(ups_context *ctx, const ups_geom *g, const float *xyz_d, int64_t n, int32_t *i_d,
                              int32_t *j_d, void *stream) {
    UPS_REQUIRE(ctx, "context is null");
    UPS_REQUIRE(n >= 0 && n <= ((int64_t)1 << 31) - kBlock, "n out of range");
    ups_status st;
    if (n > 0) {
        if ((st = check_ptr(xyz_d, 4, "points")) != UPS_OK) return st;
        if ((st = check_ptr(i_d, 4, "rows")) != UPS_OK) return st;
        if ((st = check_ptr(j_d, 4, "cols")) != UPS_OK) return st;
    }
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    DGeom d;
    if ((st = device_geom(ctx, g, 0, (hipStream_t)stream, &d)) != UPS_OK) return st;
    return launch_project_points(d, xyz_d, n, i_d, j_d, (hipStream_t)stream);
}

ups_status ups_normal_equations(ups_context *ctx, const ups_geom *scan_g, const float *scan_surfel_d,
                                const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *T_d, float d_max,
                                float cos_theta_max, int32_t precision, ups_normal_eq *out_d, void *stream) {
    UPS_REQUIRE(ctx, "context is null");
    ups_status st;
    if ((st = check_ptr(scan_surfel_d, 16, "scan surfel")) != UPS_OK) return st;
    if ((st = check_ptr(kf_surfel_d, 16, "keyframe surfel")) != UPS_OK) return st;
    if ((st = check_ptr(T_d, 8, "pose")) != UPS_OK) return st;
    if ((st = check_ptr(out_d, 8, "out")) != UPS_OK) return st;
    UPS_REQUIRE(d_max > 0.f, "d_max must be > 0");
    UPS_REQUIRE(precision >= UPS_PREC_KAHAN_F64 && precision <= UPS_PREC_F64, "unknown precision mode");
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    if ((int64_t)scan_g->rows * scan_g->cols > ctx->max_pixels) {
        set_error("panorama larger than the context's max_pixels");
        return UPS_ERR_WORKSPACE;
    }
    Inst I;
    memset(&I, 0, sizeof(I));
    if ((st = device_geom(ctx, scan_g, 0, (hipStream_t)stream, &I.sg[0])) != UPS_OK) return st;
    if ((st = device_geom(ctx, kf_g, 0, (hipStream_t)stream, &I.kg[0])) != UPS_OK) return st;
    I.scan[0] = (const float4 *)scan_surfel_d;
    I.kf[0] = (const float4 *)kf_surfel_d;
    I.state = ctx->state;
    I.xsync = xsync_of(ctx->state);
    I.partials = ctx->partials;
    I.pstride = (int)ctx->max_partial_blocks;
    I.neq = out_d;
    return launch_eval(I, T_d, d_max, cos_theta_max, precision, (hipStream_t)stream);
}

}  // extern "C"
