// Autotuner for the batched Gauss-Newton launches (C ABI: ups_autotune).
//
// For each panorama size it builds a synthetic batch -- every registration a
// 20 x 10 x 4 m box room seen from its centre, registered against itself at
// the identity, so every pixel is an inlier (the most expensive path) and the
// update is exactly zero -- and times the Gauss-Newton launch (update + solve
// + association + reduction) with HIP events at 1, 2, 4, 8 and 16 pixels per
// thread.
// The fastest choice per size is kept in the context (ups_batch_create uses
// it) and written to a small JSON cache keyed by the GPU architecture; a cache
// for the same architecture is loaded instead of measuring again.
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "ups_icp.hpp"

namespace ups {

int autotuned_k(ups_context *ctx, int64_t npix) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    int best = 0;
    int64_t bd = 0;
    for (const auto &e : ctx->tuned) {
        const int64_t d = e.first > npix ? e.first - npix : npix - e.first;
        if (best == 0 || d < bd) {
            best = e.second;
            bd = d;
        }
    }
    return best;
}

namespace {

__global__ void k_room(float4 *s, int rows, int cols, const float2 *lut_row, const float2 *lut_col, int copies) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = (int64_t)rows * cols;
    if (t >= n * copies) return;
    const int p = (int)(t % n);
    const int i = p / cols, j = p - i * cols;
    const float2 e = lut_row[i], a = lut_col[j];
    const float u[3] = {e.x * a.x, e.x * a.y, e.y};
    const float half[3] = {10.f, 5.f, 2.f};
    float best = 1e30f;
    int ax = 0;
    for (int k = 0; k < 3; k++) {
        const float d = fabsf(u[k]) > 0.f ? half[k] / fabsf(u[k]) : 1e30f;
        if (d < best) {
            best = d;
            ax = k;
        }
    }
    float4 o = make_float4(0.f, 0.f, 0.f, best);
    const float sg = u[ax] > 0.f ? -1.f : 1.f;
    if (ax == 0) o.x = sg;
    else if (ax == 1) o.y = sg;
    else o.z = sg;
    s[t] = o;
}

std::string arch_name(int dev) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string s = prop.gcnArchName;
    const size_t c = s.find(':');
    return c == std::string::npos ? s : s.substr(0, c);
}

bool load_cache(const std::string &path, const std::string &arch, std::vector<std::pair<int64_t, int>> &out) {
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string txt = ss.str();
    if (txt.find("\"arch\": \"" + arch + "\"") == std::string::npos) return false;
    size_t pos = 0;
    while ((pos = txt.find("\"npix\":", pos)) != std::string::npos) {
        int64_t npix = 0;
        int K = 0;
        if (sscanf(txt.c_str() + pos, "\"npix\": %ld, \"k\": %d", &npix, &K) == 2 && npix > 0 &&
            K >= 1 && K <= 64 && (K & (K - 1)) == 0)
            out.emplace_back(npix, K);
        pos += 7;
    }
    return !out.empty();
}

}  // namespace
}  // namespace ups

using namespace ups;

extern "C" ups_status ups_autotune(ups_context *ctx, const char *cache_json_path) {
    UPS_REQUIRE(ctx, "context is null");
    int prev = -1;
    UPS_CHECK_HIP(hipGetDevice(&prev));
    if (prev != ctx->device) UPS_CHECK_HIP(hipSetDevice(ctx->device));
    struct Restore {
        int d;
        ~Restore() {
            if (d >= 0) (void)hipSetDevice(d);
        }
    } restore{prev};
    const std::string arch = arch_name(ctx->device);
    std::vector<std::pair<int64_t, int>> entries;
    if (cache_json_path && load_cache(cache_json_path, arch, entries)) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->tuned = entries;
        return UPS_OK;
    }
    // measure: sizes of the lidar panoramas and their pyramid levels
    const int sizes[][2] = {{16, 128}, {32, 256}, {64, 512}, {64, 1024}, {128, 1024}, {128, 2048}};
    const int Ks[7] = {1, 2, 4, 8, 16, 32, 64};
    std::ostringstream js;
    js << "{\"arch\": \"" << arch << "\", \"kernel\": \"gauss-newton iteration, batched\", \"entries\": [";
    hipStream_t s;
    UPS_CHECK_HIP(hipStreamCreate(&s));
    hipEvent_t e0, e1;
    UPS_CHECK_HIP(hipEventCreate(&e0));
    UPS_CHECK_HIP(hipEventCreate(&e1));
    bool first = true;
    ups_status result = UPS_OK;
    for (const auto &sz : sizes) {
        const int rows = sz[0], cols = sz[1];
        const int64_t npix = (int64_t)rows * cols;
        const int copies = (int)std::max<int64_t>(1, std::min<int64_t>(256, ((int64_t)8 << 20) / npix));
        ups_geom g{rows, cols, 0.39, 0.78 / (rows - 1), 0.0, 50.0};
        DGeom dg;
        if ((result = device_geom(ctx, &g, 0, nullptr, &dg)) != UPS_OK) break;
        float4 *surf = nullptr;
        Inst *d_inst = nullptr;
        int *d_start = nullptr;
        RegState *state = nullptr;
        double *part = nullptr;
        const int pstride = (int)partial_stride((npix + kBlock - 1) / kBlock);
        hipError_t e = hipMalloc(&surf, npix * copies * sizeof(float4));
        if (e == hipSuccess) e = hipMalloc(&d_inst, copies * sizeof(Inst));
        if (e == hipSuccess) e = hipMalloc(&d_start, (copies + 1) * sizeof(int));
        if (e == hipSuccess) e = hipMalloc(&state, 2 * copies * sizeof(RegState));
        if (e == hipSuccess) e = hipMalloc(&part, (size_t)copies * 2 * pstride * kPartialStride * sizeof(double));
        if (e == hipSuccess) e = hipMemset(state, 0, 2 * copies * sizeof(RegState));
        if (e != hipSuccess) {
            set_error(std::string("autotune allocation failed: ") + hipGetErrorString(e));
            result = UPS_ERR_HIP;
        }
        int bestK = 0;
        float best = 0.f;
        std::ostringstream times;
        for (int ki = 0; ki < 7 && result == UPS_OK; ki++) {
            const int K = Ks[ki];
            const int nb = (int)((npix + kBlock * K - 1) / (kBlock * K));
            if (nb > 256) {
                times << (ki ? ", " : "") << "null";
                continue;
            }
            hipLaunchKernelGGL(k_room, dim3((unsigned)((npix * copies + 255) / 256)), dim3(256), 0, s, surf, rows,
                               cols, dg.lut_row, dg.lut_col, copies);
            std::vector<Inst> hi(copies);
            std::vector<int> start(copies + 1, 0);
            for (int c = 0; c < copies; c++) {
                Inst &I = hi[c];
                memset(&I, 0, sizeof(I));
                I.sg[0] = I.kg[0] = dg;
                I.scan[0] = I.kf[0] = surf + (size_t)c * npix;
                I.state = state + 2 * c;
                I.partials = part + (size_t)c * 2 * pstride * kPartialStride;
                I.pstride = pstride;
                I.nblocks[0] = nb;
                start[c + 1] = start[c] + nb;
            }
            e = hipMemcpy(d_inst, hi.data(), copies * sizeof(Inst), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(d_start, start.data(), (copies + 1) * sizeof(int), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                set_error(std::string("autotune upload failed: ") + hipGetErrorString(e));
                result = UPS_ERR_HIP;
                break;
            }
            // identity initial poses
            std::vector<ups_pose> hp(copies);
            for (auto &P : hp) {
                memset(&P, 0, sizeof(P));
                P.R[0] = P.R[4] = P.R[8] = 1.0;
            }
            ups_pose *d_init = nullptr;
            int *d_pre = nullptr;
            e = hipMalloc(&d_init, copies * sizeof(ups_pose));
            if (e == hipSuccess) e = hipMalloc(&d_pre, (copies + 1) * sizeof(int));
            if (e == hipSuccess) e = hipMemcpy(d_init, hp.data(), copies * sizeof(ups_pose), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemset(d_pre, 0, (copies + 1) * sizeof(int));
            if (e != hipSuccess) {
                set_error(std::string("autotune upload failed: ") + hipGetErrorString(e));
                result = UPS_ERR_HIP;
                (void)hipFree(d_init);
                (void)hipFree(d_pre);
                break;
            }
            result = launch_prepare_batch(d_inst, d_init, copies, 1, d_pre, 0, nullptr, nullptr, s);
            StepArgs a;
            memset(&a, 0, sizeof(a));
            a.level = 0;
            a.prev_level = -1;
            a.d_max2 = 0.25f;
            a.cos_theta = 0.866f;
            a.min_inliers = 1;
            const int reps = 20;
            for (int r = 0; r < reps + 3 && result == UPS_OK; r++) {
                if (r == 3) (void)hipEventRecord(e0, s);
                a.parity = r & 1;
                a.first_of_level = (r == 0);
                result = launch_icp_batch(K, UPS_PREC_KAHAN_F64, MODE_ITER, d_inst, d_start, copies, a,
                                          start[copies], s);
                a.prev_level = 0;
            }
            if (result == UPS_OK) (void)hipEventRecord(e1, s);
            (void)hipStreamSynchronize(s);
            (void)hipFree(d_init);
            (void)hipFree(d_pre);
            if (result != UPS_OK) break;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) {
                set_error(std::string("autotune run failed: ") + hipGetErrorString(e));
                result = UPS_ERR_HIP;
                break;
            }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const float us = ms * 1000.f / reps;
            times << (ki ? ", " : "") << us;
            if (bestK == 0 || us < best) {
                best = us;
                bestK = K;
            }
        }
        (void)hipFree(surf);
        (void)hipFree(d_inst);
        (void)hipFree(d_start);
        (void)hipFree(state);
        (void)hipFree(part);
        if (result != UPS_OK) break;
        entries.emplace_back(npix, bestK);
        js << (first ? "" : ",") << "\n  {\"npix\": " << npix << ", \"k\": " << bestK << ", \"rows\": " << rows
           << ", \"cols\": " << cols << ", \"batch\": " << copies << ", \"us_per_launch_k1_2_4_8_16_32_64\": ["
           << times.str() << "]}";
        first = false;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    if (result != UPS_OK) return result;
    js << "\n]}\n";
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->tuned = entries;
    }
    if (cache_json_path && cache_json_path[0]) {
        std::ofstream f(cache_json_path);
        if (!f) {
            set_error(std::string("cannot write ") + cache_json_path);
            return UPS_ERR_INVALID_ARG;
        }
        f << js.str();
    }
    return UPS_OK;
}
