// ups_register_scan_noalloc: the registration of ups_register_scan (Section
// III-B) for callers that cannot allocate device memory.  No context: the
// scratch the registration kernels need beyond their inputs and outputs --
// both panoramas' ray tables, the block partials, the two state slots and the
// one-XCD level kernels' counters -- lives in one static device array per
// GPU, `scratch`, of kScratchBytes.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol): the device
// address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch[device].
//
// Every call on a GPU uses that GPU's copy and leaves its contents behind.
// Each call writes the ray tables and the registration state before any
// kernel reads them, and a launch reads only block partials an earlier
// launch of the same call wrote.  The level counters must be zero when a call
// starts: they are zero when the code object is loaded (static storage), and
// every call's launches after the level kernel zero them again.  Calls that
// overlap in time on one GPU (two streams, two threads) race on the array.
#include <cmath>
#include <mutex>
#include <string>

#include "ups_icp.hpp"

namespace ups {
namespace {

// Largest panorama (scan or keyframe), in pixels: 128 x 2048.
constexpr int64_t kMaxPixels = 262144;
// Ray-table entries per geometry: rows + cols of any accepted geometry of at
// most kMaxPixels pixels (rows >= 2, cols <= 16384).
constexpr int64_t kMaxLut = 16384 + kMaxPixels / 16384;
// Blocks of the widest launch (pick_k_single keeps it at or below 256; the
// context sizes its partials the same way from the pixel count).
constexpr int64_t kPstride = (kMaxPixels / kBlock + 64 + 15) / 16 * 16;

constexpr int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }
constexpr int64_t kLutBytes = align256(kMaxLut * (int64_t)sizeof(float2));
constexpr int64_t kPartialBytes = align256(2 * kPartialStride * kPstride * (int64_t)sizeof(double));
constexpr int64_t kStateBytes = align256((int64_t)kSingleStateBytes);

// byte offsets of the sections
constexpr int64_t kOffLutScan = 0;
constexpr int64_t kOffLutKf = kOffLutScan + kLutBytes;
constexpr int64_t kOffPartials = kOffLutKf + kLutBytes;
constexpr int64_t kOffState = kOffPartials + kPartialBytes;
constexpr int64_t kScratchBytes = kOffState + kStateBytes;
static_assert(kScratchBytes <= (4 << 20), "the static scratch stays within 4 MiB");

constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
unsigned char *g_scratch[kMaxDevices];  // device address of each GPU's copy (null until looked up)

// The device address of the current device's copy of `scratch`.
ups_status scratch_of(int dev, unsigned char **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        UPS_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        UPS_REQUIRE(ptr != nullptr && ((uintptr_t)ptr) % 256 == 0, "static scratch has no aligned device address");
        g_scratch[dev] = (unsigned char *)ptr;
    }
    *out = g_scratch[dev];
    return UPS_OK;
}

}  // namespace

// (cos, sin) of every row elevation and column azimuth of two geometries
// (blockIdx.y = 0: scan, 1: keyframe), computed in FP64 and rounded to FP32
// exactly as the host computes the context's tables: el = el_top - i d_el,
// az = 2 pi j / cols, with no fused multiply-add.
__global__ __launch_bounds__(kBlock) void k_ray_tables(int rows_s, int cols_s, double el_top_s, double d_el_s,
                                                       float2 *out_s, int rows_k, int cols_k, double el_top_k,
                                                       double d_el_k, float2 *out_k) {
#pragma clang fp contract(off)
    const bool kf = blockIdx.y == 1;
    const int rows = kf ? rows_k : rows_s, cols = kf ? cols_k : cols_s;
    const double el_top = kf ? el_top_k : el_top_s, d_el = kf ? d_el_k : d_el_s;
    float2 *out = kf ? out_k : out_s;
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k < rows) {
        const double el = el_top - (double)k * d_el;
        out[k] = make_float2((float)cos(el), (float)sin(el));
    } else if (k < rows + cols) {
        const int j = k - rows;
        const double az = 2.0 * M_PI * (double)j / (double)cols;
        out[k] = make_float2((float)cos(az), (float)sin(az));
    }
}

}  // namespace ups

using namespace ups;

extern "C" ups_status ups_register_scan_noalloc(const ups_geom *scan_g, const float *scan_surfel_d,
                                                const ups_geom *kf_g, const float *kf_surfel_d, const ups_pose *init_d,
                                                const ups_icp_params *p, ups_icp_result *result_d, void *stream) {
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
    if ((int64_t)scan_g->rows * scan_g->cols > kMaxPixels || (int64_t)kf_g->rows * kf_g->cols > kMaxPixels) {
        set_error("ups_register_scan_noalloc: panoramas are limited to " + std::to_string(kMaxPixels) +
                  " pixels (its static scratch); use ups_register_scan with a context for larger ones");
        return UPS_ERR_WORKSPACE;
    }
    int dev = -1;
    UPS_CHECK_HIP(hipGetDevice(&dev));
    UPS_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
    if (stream) {
        hipDevice_t sdev = -1;
        UPS_CHECK_HIP(hipStreamGetDevice((hipStream_t)stream, &sdev));
        UPS_REQUIRE(sdev == dev, "the stream belongs to another device than the current one");
    }
    unsigned char *base = nullptr;
    if ((st = scratch_of(dev, &base)) != UPS_OK) return st;
    float2 *lut_s = (float2 *)(base + kOffLutScan), *lut_k = (float2 *)(base + kOffLutKf);

    const int nmax = std::max(scan_g->rows + scan_g->cols, kf_g->rows + kf_g->cols);
    hipLaunchKernelGGL(k_ray_tables, dim3((nmax + kBlock - 1) / kBlock, 2), dim3(kBlock), 0, (hipStream_t)stream,
                       scan_g->rows, scan_g->cols, scan_g->el_top, scan_g->d_el, lut_s, kf_g->rows, kf_g->cols,
                       kf_g->el_top, kf_g->d_el, lut_k);
    UPS_CHECK_HIP(hipGetLastError());

    Inst I;
    memset(&I, 0, sizeof(I));
    for (int l = 0; l < p->levels; l++) {
        I.sg[l] = geom_view(scan_g, l, lut_s, lut_s + scan_g->rows);
        I.kg[l] = geom_view(kf_g, l, lut_k, lut_k + kf_g->rows);
        // every level is read from the level-0 images
        I.scan[l] = (const float4 *)scan_surfel_d;
        I.kf[l] = (const float4 *)kf_surfel_d;
    }
    I.state = (RegState *)(base + kOffState);
    I.xsync = xsync_of(I.state);
    I.partials = (double *)(base + kOffPartials);
    I.pstride = (int)kPstride;
    I.res = result_d;
    return launch_register(I, init_d, *p, (hipStream_t)stream);
}
