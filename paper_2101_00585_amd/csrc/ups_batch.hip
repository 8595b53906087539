// Batches of independent registrations (C ABI: ups_batch_*, ups_register_batch).
//
// Planning (ups_batch_create) lays out every registration's descriptor, its
// pyramid levels, two state slots and two partial buffers in device memory,
// plus one prefix table of tile counts per pyramid level and the persistent
// scheduler's ticket map.  A call (ups_register_batch) starts with one prepare
// launch (states and pyramids of all registrations), then runs the
// Gauss-Newton iterations under one of two schedulers:
//   launches: per iteration one launch over every tile of the level, each
//     block first applying its registration's pending update (blocks of
//     registrations that stopped exit at once);
//   persistent: the scheduler's set-up (the first job of every registration)
//     and one persistent launch in which every registration advances through
//     its iterations independently of the others (k_icp_persistent; a
//     registration whose level converged or that failed publishes no further
//     iterations, so the launch's work follows the active registrations);
// and ends with the evaluation launch at the final poses and the finish
// launch that writes the results.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ups_icp.hpp"

using namespace ups;

struct ups_batch {
    int device = 0;
    int n = 0;
    ups_icp_params p;       // p.iters: the schedule of ups_register_batch calls (ups_batch_set_iterations)
    int iters_full[4] = {0, 0, 0, 0};  // the schedule the batch was created with (the fallback's)
    int K[4] = {1, 1, 1, 1};
    int total_tiles[4] = {0, 0, 0, 0};
    int total_pre = 0;
    Inst *d_inst = nullptr;       // [n]
    int *d_tile_start = nullptr;  // [4][n+1]
    unsigned *d_tile_of = nullptr;  // per level, (registration << 16) | tile of each tile (StepArgs::tile_of)
    int64_t tile_of_off[4] = {0, 0, 0, 0};
    int *d_pre_start = nullptr;   // [n+1]
    float4 *pyr = nullptr;
    RegState *state = nullptr;    // [n][2]
    double *partials = nullptr;   // [n][2][kPartialStride][pstride]
    // batched normals
    NormImg *d_nimg = nullptr;
    unsigned *d_ntile_of = nullptr;  // [total_ntiles]: (image << kNormTileBits) | tile
    float4 *ntmp = nullptr;
    int n_nimg = 0, total_ntiles = 0;
    // identity-started fallback
    ups_pose *ident = nullptr;       // [n] identity poses
    uint8_t *mask = nullptr;         // [n] registrations the fallback reruns
    ups_icp_result *alt = nullptr;   // [n] fallback results
    Compact *comp = nullptr;         // the registrations the fallback reruns ...
    int *comp_list = nullptr;        // ... [n]
    int *comp_start = nullptr;       // ... and their tile prefix tables [4][n+1] (subset tiles)
    // the fallback's launches over a subset tile each level with as few pixels
    // per thread as keep every registration within 256 tiles (a subset is
    // small: more, shorter tiles), with descriptors and partial buffers of
    // their own (the states are the batch's)
    int Ks[4] = {1, 1, 1, 1};
    int total_tiles_sub[4] = {0, 0, 0, 0};
    Inst *d_inst_sub = nullptr;        // [n]
    int *d_tile_start_sub = nullptr;   // [4][n+1]
    double *partials_sub = nullptr;    // [n][2][kPartialStride][pstride of the subset tiles]
    int scheduler = UPS_SCHED_LAUNCHES;
    // where the pyramid levels are built (UPS_PYR_*); in UPS_PYR_IN_NORMALS
    // mode the normals' last pass writes those of the images it computes, and
    // register / grid-search calls build only the others (need[k]: bit 0 the
    // scan, bit 1 the keyframe has no depth)
    int pyr_mode = UPS_PYR_IN_REGISTER;
    uint8_t *d_need = nullptr;           // [n]
    int *d_pre_need_start = nullptr;     // [n+1] prefix table of those images' level-1 pixels
    int total_pre_need = 0;
    // persistent scheduler
    int Kp = 0;                       // the persistent kernel's pixels per thread (the largest of kpt)
    int kpt[4] = {1, 1, 1, 1};        // pixels per thread of its tiles at each level
    int grid = 0;                     // its resident blocks
    int map_size = 0;                 // tickets of a call, at most
    Sched *sched = nullptr;
    unsigned long long *tile_map = nullptr;  // [map_size]
    SchedJob *jobs = nullptr;                // [n]
    int *arrived = nullptr;                  // [n]
};

// Grid of the launches over a subset of the batch (the fallback): they stride
// over the subset's tiles (its registrations, for the results), so that they
// cost little when it is small.
constexpr int kListBlocks = 512, kListFinishBlocks = 32;

namespace {


void free_batch(ups_batch *b) {
    (void)hipFree(b->d_inst);
    (void)hipFree(b->d_tile_start);
    (void)hipFree(b->d_tile_of);
    (void)hipFree(b->d_pre_start);
    (void)hipFree(b->pyr);
    (void)hipFree(b->state);
    (void)hipFree(b->partials);
    (void)hipFree(b->d_nimg);
    (void)hipFree(b->d_ntile_of);
    (void)hipFree(b->ntmp);
    (void)hipFree(b->ident);
    (void)hipFree(b->mask);
    (void)hipFree(b->alt);
    (void)hipFree(b->comp);
    (void)hipFree(b->d_inst_sub);
    (void)hipFree(b->d_tile_start_sub);
    (void)hipFree(b->partials_sub);
    (void)hipFree(b->sched);
    (void)hipFree(b->tile_map);
    (void)hipFree(b->jobs);
    (void)hipFree(b->arrived);
    (void)hipFree(b->d_need);
    (void)hipFree(b->d_pre_need_start);
    delete b;
}

// Library choice of pixels per thread for batch launches: the autotuned value
// if one was recorded for this size, else 8.
int default_k(ups_context *ctx, int64_t npix) {
    const int tuned = autotuned_k(ctx, npix);
    return tuned > 0 ? tuned : 8;
}

// The pyramids a register / grid-search call builds: every image's, or in
// UPS_PYR_IN_NORMALS mode those of the images without depth (the normals
// write the others): prefix table of their level-1 pixels, its total, and
// the per-registration selection (null: every image).
struct PyrWork {
    const int *start;
    int total;
    const uint8_t *need;
};
PyrWork pyramid_work(const ups_batch *b) {
    if (b->pyr_mode == UPS_PYR_IN_NORMALS) return PyrWork{b->d_pre_need_start, b->total_pre_need, b->d_need};
    return PyrWork{b->d_pre_start, b->total_pre, nullptr};
}

}  // namespace

extern "C" {

ups_status ups_batch_create(ups_context *ctx, int32_t n, const ups_batch_item *items, const ups_icp_params *p,
                            int32_t pixels_per_thread, ups_batch **out) {
    UPS_REQUIRE(ctx && items && p && out, "null argument");
    *out = nullptr;
    UPS_REQUIRE(n >= 1 && n <= ctx->max_batch, "n must be in [1, the context's max_batch]");
    UPS_REQUIRE(n <= 65535, "a batch holds at most 65535 registrations");
    UPS_REQUIRE(pixels_per_thread == 0 || (pixels_per_thread <= 64 && (pixels_per_thread & (pixels_per_thread - 1)) == 0),
                "pixels_per_thread must be 0 or a power of two up to 64");
    {
        const ups_status pst = check_icp_params(p);
        if (pst != UPS_OK) return pst;
    }
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    const int L = p->levels, s = 1 << (L - 1);
    int64_t total_scan = 0, total_kf = 0, max_npix = 0;
    for (int k = 0; k < n; k++) {
        const ups_batch_item &it = items[k];
        UPS_REQUIRE(it.scan_surfel_d && it.kf_surfel_d, "item " + std::to_string(k) + ": surfel pointers are null");
        UPS_REQUIRE(((uintptr_t)it.scan_surfel_d % 16) == 0 && ((uintptr_t)it.kf_surfel_d % 16) == 0,
                    "item " + std::to_string(k) + ": surfel images must be 16-byte aligned");
        for (const ups_geom *g : {&it.scan_g, &it.kf_g}) {
            UPS_REQUIRE(g->rows % s == 0 && g->rows / s >= 2 && g->cols % (64 * s) == 0,
                        "item " + std::to_string(k) + ": rows/cols not divisible for the pyramid");
        }
        total_scan += (int64_t)it.scan_g.rows * it.scan_g.cols;
        total_kf += (int64_t)it.kf_g.rows * it.kf_g.cols;
        max_npix = std::max(max_npix, (int64_t)it.scan_g.rows * it.scan_g.cols);
    }
    if (total_scan > ctx->max_batch_pixels || total_kf > ctx->max_batch_pixels) {
        set_error("batch panoramas exceed the context's max_batch_pixels");
        return UPS_ERR_WORKSPACE;
    }
    ups_batch *b = new ups_batch();
    b->device = ctx->device;
    b->n = n;
    b->p = *p;
    for (int l = 0; l < 4; l++) b->iters_full[l] = p->iters[l];
    for (int l = 0; l < L; l++) {
        int K = pixels_per_thread ? pixels_per_thread : default_k(ctx, max_npix >> (2 * l));
        // every registration must fit in 256 tiles at every level
        while (K < 64 && ((max_npix >> (2 * l)) + kBlock * K - 1) / (kBlock * K) > 256) K *= 2;
        if (((max_npix >> (2 * l)) + kBlock * K - 1) / (kBlock * K) > 256) {
            free_batch(b);
            set_error("a batch panorama is too large for 256 tiles of 64 pixels per thread");
            return UPS_ERR_INVALID_ARG;
        }
        b->K[l] = K;
    }
    for (int l = 0; l < L; l++) {
        int K = 1;
        while (K < b->K[l] && ((max_npix >> (2 * l)) + kBlock * K - 1) / (kBlock * K) > 256) K *= 2;
        b->Ks[l] = K;
    }
    // the persistent kernel is compiled for the largest of these and tiles
    // each level with its own (at least a pixel group of the kernel, 4), so
    // no level has more tiles than the partial buffers hold
    for (int l = 0; l < L; l++) b->Kp = std::max(b->Kp, b->K[l]);
    for (int l = 0; l < L; l++) b->kpt[l] = std::max(b->K[l], std::min(b->Kp, 4));
    b->grid = persistent_grid(b->Kp, p->precision, p->irls_delta > 0.f);
    if (b->grid < 1) {
        free_batch(b);
        set_error("no resident blocks for the persistent batch kernel");
        return UPS_ERR_HIP;
    }

    // host descriptors
    std::vector<Inst> hi(n);
    std::vector<int> tile_start(4 * (n + 1), 0), tile_start_sub(4 * (n + 1), 0), pre_start(n + 1, 0);
    std::vector<int> pre_need_start(n + 1, 0);
    std::vector<uint8_t> need(n, 0);
    std::vector<int> nblocks_sub(4 * (size_t)n, 0);
    int64_t pyr_total = 0;
    int pstride = 1, pstride_sub = 1;
    std::vector<int64_t> pyr_off_s(n), pyr_off_k(n);
    for (int k = 0; k < n; k++) {
        const ups_batch_item &it = items[k];
        Inst &I = hi[k];
        memset(&I, 0, sizeof(I));
        int pre = 0;
        for (int l = 0; l < L; l++) {
            ups_status st;
            if ((st = device_geom(ctx, &it.scan_g, l, nullptr, &I.sg[l])) != UPS_OK ||
                (st = device_geom(ctx, &it.kf_g, l, nullptr, &I.kg[l])) != UPS_OK) {
                free_batch(b);
                return st;
            }
            const int np = I.sg[l].rows * I.sg[l].cols;
            I.nblocks[l] = (np + kBlock * b->K[l] - 1) / (kBlock * b->K[l]);
            pstride = std::max(pstride, I.nblocks[l]);
            nblocks_sub[4 * k + l] = (np + kBlock * b->Ks[l] - 1) / (kBlock * b->Ks[l]);
            pstride_sub = std::max(pstride_sub, nblocks_sub[4 * k + l]);
            if (l == 1) {
                pre += np + I.kg[l].rows * I.kg[l].cols;
                need[k] = (uint8_t)((it.scan_depth_d ? 0 : 1) | (it.kf_depth_d ? 0 : 2));
                pre_need_start[k + 1] = (need[k] & 1 ? np : 0) + (need[k] & 2 ? I.kg[l].rows * I.kg[l].cols : 0);
            }
        }
        pre_need_start[k + 1] += pre_need_start[k];
        pyr_off_s[k] = pyr_total;
        for (int l = 1; l < L; l++) pyr_total += (int64_t)I.sg[l].rows * I.sg[l].cols;
        pyr_off_k[k] = pyr_total;
        for (int l = 1; l < L; l++) pyr_total += (int64_t)I.kg[l].rows * I.kg[l].cols;
        pre_start[k + 1] = pre_start[k] + pre;
    }
    for (int l = 0; l < 4; l++) {
        for (int k = 0; k < n; k++)
            tile_start[l * (n + 1) + k + 1] = tile_start[l * (n + 1) + k] + (l < L ? hi[k].nblocks[l] : 0);
        b->total_tiles[l] = tile_start[l * (n + 1) + n];
        for (int k = 0; k < n; k++)
            tile_start_sub[l * (n + 1) + k + 1] = tile_start_sub[l * (n + 1) + k] + nblocks_sub[4 * k + l];
        b->total_tiles_sub[l] = tile_start_sub[l * (n + 1) + n];
    }
    b->total_pre = pre_start[n];
    b->total_pre_need = pre_need_start[n];
    // tickets of a call, at most: every iteration of every level of every
    // registration, plus the last ticket of each block
    {
        int64_t tickets = b->grid + 64;
        for (int k = 0; k < n; k++) {
            for (int l = 0; l < L; l++) {
                const int64_t np = (int64_t)hi[k].sg[l].rows * hi[k].sg[l].cols;
                const int64_t t = (np + kBlock * b->kpt[l] - 1) / (kBlock * b->kpt[l]);
                tickets += t * p->iters[l];
            }
        }
        if (tickets > (int64_t)1 << 30) {
            free_batch(b);
            set_error("batch too large for the scheduler's ticket map");
            return UPS_ERR_INVALID_ARG;
        }
        b->map_size = (int)tickets;
    }

    // batched-normals images: every scan / keyframe with a depth pointer
    std::vector<NormImg> nimg;
    std::vector<std::pair<int, int>> nimg_of;  // (registration, 0 scan / 1 keyframe) of each entry
    std::vector<unsigned> ntile_of;
    int64_t ntmp_total = 0;
    for (int k = 0; k < n; k++) {
        const ups_batch_item &it = items[k];
        if (it.scan_depth_d) {
            nimg.push_back(NormImg{hi[k].sg[0], it.scan_depth_d, (float4 *)it.scan_surfel_d, nullptr, {}});
            nimg_of.emplace_back(k, 0);
            ntmp_total += (int64_t)hi[k].sg[0].rows * hi[k].sg[0].cols;
        }
        if (it.kf_depth_d) {
            nimg.push_back(NormImg{hi[k].kg[0], it.kf_depth_d, (float4 *)it.kf_surfel_d, nullptr, {}});
            nimg_of.emplace_back(k, 1);
            ntmp_total += (int64_t)hi[k].kg[0].rows * hi[k].kg[0].cols;
        }
    }

    hipError_t e = hipSuccess;
    auto alloc = [&](void **ptr, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(ptr, bytes > 0 ? bytes : 16);
    };
    alloc((void **)&b->d_inst, n * sizeof(Inst));
    alloc((void **)&b->d_tile_start, tile_start.size() * sizeof(int));
    // block -> (registration, tile) of every level, so that a block finds its
    // tile with one load
    std::vector<unsigned> tile_of;
    for (int l = 0; l < 4; l++) {
        b->tile_of_off[l] = (int64_t)tile_of.size();
        for (int k = 0; k < n; k++)
            for (int t = tile_start[l * (n + 1) + k]; t < tile_start[l * (n + 1) + k + 1]; t++)
                tile_of.push_back(((unsigned)k << 16) | (unsigned)(t - tile_start[l * (n + 1) + k]));
    }
    alloc((void **)&b->d_tile_of, std::max<size_t>(tile_of.size(), 1) * sizeof(unsigned));
    alloc((void **)&b->d_pre_start, pre_start.size() * sizeof(int));
    alloc((void **)&b->pyr, std::max<int64_t>(pyr_total, 1) * sizeof(float4));
    alloc((void **)&b->state, (size_t)n * 2 * sizeof(RegState));
    pstride = (int)partial_stride(pstride);
    alloc((void **)&b->partials, (size_t)n * 2 * pstride * kPartialStride * sizeof(double));
    alloc((void **)&b->ident, (size_t)n * sizeof(ups_pose));
    alloc((void **)&b->mask, (size_t)n);
    alloc((void **)&b->alt, (size_t)n * sizeof(ups_icp_result));
    alloc((void **)&b->comp, sizeof(Compact) + ((size_t)n + 4 * ((size_t)n + 1)) * sizeof(int) + 64);
    alloc((void **)&b->d_inst_sub, n * sizeof(Inst));
    alloc((void **)&b->d_tile_start_sub, tile_start_sub.size() * sizeof(int));
    pstride_sub = (int)partial_stride(pstride_sub);
    alloc((void **)&b->partials_sub, (size_t)n * 2 * pstride_sub * kPartialStride * sizeof(double));
    alloc((void **)&b->sched, sizeof(Sched));
    alloc((void **)&b->tile_map, (size_t)b->map_size * sizeof(unsigned long long));
    alloc((void **)&b->jobs, (size_t)n * sizeof(SchedJob));
    alloc((void **)&b->arrived, (size_t)n * sizeof(int));
    alloc((void **)&b->d_need, (size_t)n);
    alloc((void **)&b->d_pre_need_start, pre_need_start.size() * sizeof(int));
    if (e == hipSuccess) {
        b->comp_list = (int *)((char *)b->comp + 64);
        b->comp_start = b->comp_list + n;
    }
    if (e == hipSuccess) {
        std::vector<ups_pose> id(n);
        for (ups_pose &q : id) {
            memset(&q, 0, sizeof(q));
            q.R[0] = q.R[4] = q.R[8] = 1.0;
        }
        e = hipMemcpy(b->ident, id.data(), n * sizeof(ups_pose), hipMemcpyHostToDevice);
    }
    if (!nimg.empty()) {
        alloc((void **)&b->d_nimg, nimg.size() * sizeof(NormImg));
        alloc((void **)&b->ntmp, ntmp_total * sizeof(float4));
    }
    if (e != hipSuccess) {
        free_batch(b);
        set_error(std::string("batch allocation failed: ") + hipGetErrorString(e));
        return UPS_ERR_HIP;
    }
    for (int k = 0; k < n; k++) {
        Inst &I = hi[k];
        I.scan[0] = (const float4 *)items[k].scan_surfel_d;
        I.kf[0] = (const float4 *)items[k].kf_surfel_d;
        int64_t os = pyr_off_s[k], ok = pyr_off_k[k];
        for (int l = 1; l < L; l++) {
            I.scan[l] = b->pyr + os;
            os += (int64_t)I.sg[l].rows * I.sg[l].cols;
            I.kf[l] = b->pyr + ok;
            ok += (int64_t)I.kg[l].rows * I.kg[l].cols;
        }
        I.state = b->state + 2 * k;
        I.partials = b->partials + (size_t)k * 2 * pstride * kPartialStride;
        I.pstride = pstride;
    }
    if (!nimg.empty()) {
        int64_t off = 0;
        for (size_t m = 0; m < nimg.size(); m++) {
            NormImg &im = nimg[m];
            const Inst &I = hi[nimg_of[m].first];
            for (int l = 1; l <= 3; l++)
                im.pyr[l - 1] = l < L ? (float4 *)(nimg_of[m].second == 0 ? I.scan[l] : I.kf[l]) : nullptr;
            im.tmp = b->ntmp + off;
            off += (int64_t)im.g.rows * im.g.cols;
            const int nt = normal_tiles(im.g);
            if (nt >= (1 << kNormTileBits)) {
                free_batch(b);
                set_error("panorama with too many normal tiles for a batch (at most 8191 tiles of 64 x 16 pixels)");
                return UPS_ERR_INVALID_ARG;
            }
            for (int t = 0; t < nt; t++) ntile_of.push_back(((unsigned)m << kNormTileBits) | (unsigned)t);
        }
        b->n_nimg = (int)nimg.size();
        b->total_ntiles = (int)ntile_of.size();
        alloc((void **)&b->d_ntile_of, ntile_of.size() * sizeof(unsigned));
    }
    if (e == hipSuccess) e = hipMemcpy(b->d_inst, hi.data(), n * sizeof(Inst), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        std::vector<Inst> hs(hi);
        for (int k = 0; k < n; k++) {
            for (int l = 0; l < 4; l++) hs[k].nblocks[l] = nblocks_sub[4 * k + l];
            hs[k].partials = b->partials_sub + (size_t)k * 2 * pstride_sub * kPartialStride;
            hs[k].pstride = pstride_sub;
        }
        e = hipMemcpy(b->d_inst_sub, hs.data(), n * sizeof(Inst), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
        e = hipMemcpy(b->d_tile_start_sub, tile_start_sub.data(), tile_start_sub.size() * sizeof(int),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_tile_start, tile_start.data(), tile_start.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && !tile_of.empty())
        e = hipMemcpy(b->d_tile_of, tile_of.data(), tile_of.size() * sizeof(unsigned), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_pre_start, pre_start.data(), pre_start.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_pre_need_start, pre_need_start.data(), pre_need_start.size() * sizeof(int),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->d_need, need.data(), (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(b->state, 0, (size_t)n * 2 * sizeof(RegState));
    if (e == hipSuccess) e = hipMemset(b->sched, 0, sizeof(Sched));  // epoch 0: no ticket carries a tile yet
    if (e == hipSuccess) e = hipMemset(b->tile_map, 0, (size_t)b->map_size * sizeof(unsigned long long));
    if (e == hipSuccess && !nimg.empty()) {
        e = hipMemcpy(b->d_nimg, nimg.data(), nimg.size() * sizeof(NormImg), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(b->d_ntile_of, ntile_of.data(), ntile_of.size() * sizeof(unsigned), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_batch(b);
        set_error(std::string("batch upload failed: ") + hipGetErrorString(e));
        return UPS_ERR_HIP;
    }
    *out = b;
    return UPS_OK;
}

void ups_batch_destroy(ups_batch *b) {
    if (!b) return;
    DeviceGuard dg(b->device);
    free_batch(b);
}

ups_status ups_batch_time_iteration(ups_context *ctx, ups_batch *b, int32_t level, int32_t n_launches, void *stream,
                                    float *us_per_launch) {
    UPS_REQUIRE(ctx && b && us_per_launch, "null argument");
    UPS_REQUIRE(level >= 0 && level < b->p.levels, "level out of range");
    UPS_REQUIRE(n_launches >= 1 && n_launches <= 10000, "n_launches must be in [1, 10000]");
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    hipStream_t s = (hipStream_t)stream;
    ups ::StepArgs a;
    memset(&a, 0, sizeof(a));
    a.level = level;
    a.prev_level = -1;
    a.d_max2 = b->p.d_max[level] * b->p.d_max[level];
    a.cos_theta = b->p.cos_theta_max;
    a.irls_delta = b->p.irls_delta;
    a.min_inliers = b->p.min_inliers;
    a.tile_of = b->d_tile_of + b->tile_of_off[level];
    ups_status st;
    if ((st = launch_activate_batch(b->d_inst, b->n, s)) != UPS_OK) return st;
    hipEvent_t e0, e1;
    UPS_CHECK_HIP(hipEventCreate(&e0));
    UPS_CHECK_HIP(hipEventCreate(&e1));
    // the main loop's (fused) launch, state slot 0 in, no update pending: the
    // same tile work every launch
    st = launch_icp_batch(b->K[level], b->p.precision, MODE_ITER, b->d_inst, b->d_tile_start + level * (b->n + 1),
                          b->n, a, b->total_tiles[level], s, true);  // warm-up
    hipError_t e = hipEventRecord(e0, s);
    for (int k = 0; k < n_launches && st == UPS_OK && e == hipSuccess; k++)
        st = launch_icp_batch(b->K[level], b->p.precision, MODE_ITER, b->d_inst,
                              b->d_tile_start + level * (b->n + 1), b->n, a, b->total_tiles[level], s, true);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != UPS_OK) return st;
    UPS_CHECK_HIP(e);
    *us_per_launch = ms * 1000.f / n_launches;
    return UPS_OK;
}

ups_status ups_batch_pixels_per_thread(const ups_batch *b, int32_t out[4]) {
    UPS_REQUIRE(b && out, "null argument");
    for (int l = 0; l < 4; l++) out[l] = b->K[l];
    return UPS_OK;
}

ups_status ups_batch_set_scheduler(ups_batch *b, int32_t scheduler) {
    UPS_REQUIRE(b, "null argument");
    UPS_REQUIRE(scheduler == UPS_SCHED_LAUNCHES || scheduler == UPS_SCHED_PERSISTENT,
                "scheduler must be UPS_SCHED_LAUNCHES or UPS_SCHED_PERSISTENT");
    b->scheduler = scheduler;
    return UPS_OK;
}

ups_status ups_batch_set_pyramid_mode(ups_batch *b, int32_t mode) {
    UPS_REQUIRE(b, "null argument");
    UPS_REQUIRE(mode == UPS_PYR_IN_REGISTER || mode == UPS_PYR_IN_NORMALS,
                "mode must be UPS_PYR_IN_REGISTER or UPS_PYR_IN_NORMALS");
    b->pyr_mode = mode;
    return UPS_OK;
}

ups_status ups_batch_set_iterations(ups_batch *b, const int32_t iters[4]) {
    UPS_REQUIRE(b && iters, "null argument");
    for (int l = 0; l < b->p.levels; l++)
        UPS_REQUIRE(iters[l] >= 0 && iters[l] <= b->iters_full[l],
                    "iters[" + std::to_string(l) + "] must be in [0, " + std::to_string(b->iters_full[l]) + "]");
    for (int l = 0; l < b->p.levels; l++) b->p.iters[l] = iters[l];
    return UPS_OK;
}

ups_status ups_batch_schedule(const ups_batch *b, int32_t *blocks, int32_t kpt[4]) {
    UPS_REQUIRE(b && blocks && kpt, "null argument");
    *blocks = b->grid;
    for (int l = 0; l < 4; l++) kpt[l] = b->kpt[l];
    return UPS_OK;
}

ups_status ups_batch_normals(ups_context *ctx, ups_batch *b, const ups_normal_params *p, void *stream) {
    UPS_REQUIRE(ctx && b && p, "null argument");
    UPS_REQUIRE(p->atrous_levels >= 1 && p->atrous_levels <= 3, "batched normals need atrous_levels in [1, 3]");
    UPS_REQUIRE(p->sigma_n > 0.f && p->sigma_r > 0.f && p->max_rel_jump >= 0.f, "sigmas must be > 0");
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    if (b->n_nimg == 0) return UPS_OK;
    // in UPS_PYR_IN_NORMALS mode the last pass also writes the images' pyramids
    return launch_normals_batch(b->d_nimg, b->d_ntile_of, b->total_ntiles, *p,
                                b->pyr_mode == UPS_PYR_IN_NORMALS ? 1 : 0, (hipStream_t)stream);
}

}  // extern "C"

namespace {

// The launch sequence of a batch call over every registration: prepare, then
// one launch per Gauss-Newton iteration in which each block first applies
// its registration's pending update (state and partials in ping-pong slots),
// the evaluation launch (which applies the last update) and the finish.
ups_status register_batch_fused(ups_batch *b, const ups_pose *init_d, ups_icp_result *results_d, hipStream_t s) {
    ups_status st;
    const ups_icp_params &p = b->p;
    const int n = b->n;
    const PyrWork pw = pyramid_work(b);
    if ((st = launch_prepare_batch(b->d_inst, init_d, n, p.levels, pw.start, pw.total, nullptr, pw.need, s)) != UPS_OK)
        return st;
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.cos_theta = p.cos_theta_max;
    a.irls_delta = p.irls_delta;
    a.min_inliers = p.min_inliers;
    a.stop_norm = p.stop_update_norm;
    a.prev_level = -1;
    int parity = 0;
    for (int l = p.levels - 1; l >= 0; l--) {
        a.level = l;
        a.d_max2 = p.d_max[l] * p.d_max[l];
        a.tile_of = b->d_tile_of + b->tile_of_off[l];
        for (int it = 0; it < p.iters[l]; it++) {
            a.parity = parity;
            a.first_of_level = it == 0;
            if ((st = launch_icp_batch(b->K[l], p.precision, MODE_ITER, b->d_inst, b->d_tile_start + l * (n + 1), n,
                                       a, b->total_tiles[l], s, true)) != UPS_OK)
                return st;
            a.prev_level = l;
            parity ^= 1;
        }
    }
    a.level = 0;
    a.parity = parity;
    a.first_of_level = 0;
    a.d_max2 = p.d_max[0] * p.d_max[0];
    a.tau2 = a.d_max2;
    a.check_max_iters = (p.stop_update_norm > 0.0 && p.iters[0] > 0);
    a.tile_of = b->d_tile_of + b->tile_of_off[0];
    if ((st = launch_icp_batch(b->K[0], p.precision, MODE_EVAL, b->d_inst, b->d_tile_start, n, a, b->total_tiles[0],
                               s, true)) != UPS_OK)
        return st;
    return launch_finish_batch(p.precision, b->d_inst, n, parity ^ 1, results_d, s);
}

// A call over the masked-in registrations (the fallback): their pyramids left
// by the previous call are reused, and the launches go through the batch's
// Compact list of them, tiled with the subset's pixels per thread (Ks), in the
// main loop's fused form: prepare, one launch per Gauss-Newton iteration in
// which each tile first applies its registration's pending update, the
// evaluation launch, and the results of the listed registrations.
ups_status register_batch_subset(ups_batch *b, const ups_pose *init_d, const uint8_t *mask, ups_icp_result *results_d,
                                 hipStream_t s) {
    ups_status st;
    ups_icp_params p = b->p;  // the schedule the batch was created with
    for (int l = 0; l < 4; l++) p.iters[l] = b->iters_full[l];
    const int n = b->n;
    if ((st = launch_prepare_batch(b->d_inst, init_d, n, p.levels, b->d_pre_start, 0, mask, nullptr, s)) != UPS_OK)
        return st;
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.cos_theta = p.cos_theta_max;
    a.irls_delta = p.irls_delta;
    a.min_inliers = p.min_inliers;
    a.stop_norm = p.stop_update_norm;
    a.prev_level = -1;
    int parity = 0;
    for (int l = p.levels - 1; l >= 0; l--) {
        a.level = l;
        a.d_max2 = p.d_max[l] * p.d_max[l];
        for (int it = 0; it < p.iters[l]; it++) {
            a.parity = parity;
            a.first_of_level = it == 0;
            if ((st = launch_icp_batch_list(b->Ks[l], p.precision, MODE_ITER, b->d_inst_sub, b->comp, b->comp_list,
                                            b->comp_start + l * (n + 1), n, a,
                                            std::min(b->total_tiles_sub[l], kListBlocks), s)) != UPS_OK)
                return st;
            a.prev_level = l;
            parity ^= 1;
        }
    }
    a.level = 0;
    a.parity = parity;
    a.first_of_level = 0;
    a.d_max2 = p.d_max[0] * p.d_max[0];
    a.tau2 = a.d_max2;
    a.check_max_iters = (p.stop_update_norm > 0.0 && p.iters[0] > 0);
    if ((st = launch_icp_batch_list(b->Ks[0], p.precision, MODE_EVAL, b->d_inst_sub, b->comp, b->comp_list,
                                    b->comp_start, n, a, std::min(b->total_tiles_sub[0], kListBlocks), s)) != UPS_OK)
        return st;
    return launch_finish_batch_list(p.precision, b->d_inst_sub, b->comp, b->comp_list, std::min(n, kListFinishBlocks),
                                    parity ^ 1, results_d, s);
}

// A batch call under the persistent scheduler: prepare (states, and pyramids
// unless a mask reuses those of the previous call), the scheduler's first
// jobs (mask: only the masked-in registrations take part; the others keep
// their results), the persistent launch that runs every registration through
// its iterations, the evaluation launch and the finish launch.
ups_status register_batch_persistent(ups_batch *b, const ups_pose *init_d, const uint8_t *mask, ups_icp_result *results_d,
                               hipStream_t s) {
    ups_status st;
    const ups_icp_params &p = b->p;
    const PyrWork pw = pyramid_work(b);
    if ((st = launch_prepare_batch(b->d_inst, init_d, b->n, p.levels, pw.start, pw.total, mask, pw.need, s)) != UPS_OK)
        return st;
    SchedArgs A;
    memset(&A, 0, sizeof(A));
    A.sched = b->sched;
    A.tile_map = b->tile_map;
    A.jobs = b->jobs;
    A.arrived = b->arrived;
    A.insts = b->d_inst;
    A.results = results_d;
    A.mask = mask;
    A.n = b->n;
    A.map_size = b->map_size;
    A.levels = p.levels;
    for (int l = 0; l < 4; l++) A.kpt[l] = b->kpt[l];
    for (int l = 0; l < 4; l++) {
        // a fallback call (mask) keeps the schedule the batch was created with
        A.iters[l] = l < p.levels ? (mask ? b->iters_full[l] : p.iters[l]) : 0;
        A.d_max2[l] = l < p.levels ? p.d_max[l] * p.d_max[l] : 0.f;
    }
    A.cos_theta = p.cos_theta_max;
    A.irls_delta = p.irls_delta;
    A.min_inliers = p.min_inliers;
    A.stop_norm = p.stop_update_norm;
    if ((st = launch_sched_init(A, s)) != UPS_OK) return st;
    if ((st = launch_icp_persistent(b->Kp, p.precision, A, b->grid, s)) != UPS_OK) return st;
    // quality at the final poses: one evaluation launch over every tile of
    // level 0 (masked-out registrations leave), then one block per result
    StepArgs e;
    memset(&e, 0, sizeof(e));
    e.level = 0;
    e.prev_level = -1;
    e.d_max2 = p.d_max[0] * p.d_max[0];
    e.tau2 = e.d_max2;
    e.cos_theta = p.cos_theta_max;
    e.irls_delta = p.irls_delta;
    e.min_inliers = p.min_inliers;
    e.stop_norm = p.stop_update_norm;
    e.tile_of = b->d_tile_of + b->tile_of_off[0];
    if ((st = launch_icp_batch(b->K[0], p.precision, MODE_EVAL, b->d_inst, b->d_tile_start, b->n, e, b->total_tiles[0],
                               s)) != UPS_OK)
        return st;
    return launch_finish_batch(p.precision, b->d_inst, b->n, 0, results_d, s);
}

ups_status register_batch_impl(ups_batch *b, const ups_pose *init_d, const uint8_t *mask, ups_icp_result *results_d,
                               hipStream_t s) {
    if (b->scheduler == UPS_SCHED_PERSISTENT) return register_batch_persistent(b, init_d, mask, results_d, s);
    if (mask) return register_batch_subset(b, init_d, mask, results_d, s);
    return register_batch_fused(b, init_d, results_d, s);
}

}  // namespace

extern "C" {

ups_status ups_register_batch(ups_context *ctx, ups_batch *b, const ups_pose *init_d, ups_icp_result *results_d,
                              void *stream) {
    UPS_REQUIRE(ctx && b, "null argument");
    ups_status st;
    if ((st = check_ptr(init_d, 8, "init poses")) != UPS_OK) return st;
    if ((st = check_ptr(results_d, 8, "results")) != UPS_OK) return st;
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    return register_batch_impl(b, init_d, nullptr, results_d, (hipStream_t)stream);
}

ups_status ups_batch_grid_search(ups_context *ctx, ups_batch *b, const ups_grid_params *gp, const ups_pose *base_d,
                                  int32_t *scores_d, ups_pose *best_d, int32_t *best_score_d, void *stream) {
    UPS_REQUIRE(ctx && b && gp, "null argument");
    UPS_REQUIRE(gp->level >= 0 && gp->level < b->p.levels, "grid level must be one of the batch's pyramid levels");
    UPS_REQUIRE(gp->n_yaw >= 1 && gp->n_xy >= 1 && (int64_t)gp->n_yaw * gp->n_xy * gp->n_xy <= 65535,
                "need n_yaw, n_xy >= 1 and at most 65535 candidates");
    UPS_REQUIRE(std::isfinite(gp->xy_step) && gp->xy_step >= 0.f, "xy_step must be finite and >= 0");
    UPS_REQUIRE(gp->d_max > 0.f && std::isfinite(gp->cos_theta_max), "invalid Omega thresholds");
    ups_status st;
    if ((st = check_ptr(base_d, 8, "base poses")) != UPS_OK) return st;
    if ((st = check_ptr(scores_d, 4, "scores")) != UPS_OK) return st;
    if ((st = check_ptr(best_d, 8, "best poses")) != UPS_OK) return st;
    if (best_score_d && (st = check_ptr(best_score_d, 4, "best scores")) != UPS_OK) return st;
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    hipStream_t s = (hipStream_t)stream;
    const int n = b->n, l = gp->level;
    const PyrWork pw = pyramid_work(b);
    if (l > 0 && (st = launch_build_pyramids(b->d_inst, n, b->p.levels, pw.start, pw.total, pw.need, s)) != UPS_OK)
        return st;
    GridArgs g;
    g.level = l;
    g.n_yaw = gp->n_yaw;
    g.n_xy = gp->n_xy;
    g.C = gp->n_yaw * gp->n_xy * gp->n_xy;
    g.xy_step = gp->xy_step;
    g.d_max2 = gp->d_max * gp->d_max;
    g.cos_theta = gp->cos_theta_max;
    return launch_grid_search(b->d_inst, b->d_tile_start + l * (n + 1), n, b->K[l], b->total_tiles[l], base_d, g,
                              scores_d, best_d, best_score_d, s);
}

ups_status ups_batch_fallback_plan(ups_context *ctx, ups_batch *b, double min_inlier_ratio,
                                   const ups_icp_result *results_d, int32_t *count_d, void *stream) {
    UPS_REQUIRE(ctx && b, "null argument");
    UPS_REQUIRE(std::isfinite(min_inlier_ratio), "min_inlier_ratio must be finite");
    ups_status st;
    if ((st = check_ptr(results_d, 8, "results")) != UPS_OK) return st;
    if (count_d && (st = check_ptr(count_d, 4, "count")) != UPS_OK) return st;
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    return launch_fallback_plan(b->n, results_d, min_inlier_ratio, b->d_tile_start_sub, b->mask, b->comp,
                                b->comp_list, b->comp_start, count_d, (hipStream_t)stream);
}

ups_status ups_batch_fallback_run(ups_context *ctx, ups_batch *b, ups_icp_result *results_d, void *stream) {
    UPS_REQUIRE(ctx && b, "null argument");
    ups_status st;
    if ((st = check_ptr(results_d, 8, "results")) != UPS_OK) return st;
    DeviceGuard dg(ctx->device);
    UPS_CHECK_HIP(dg.err);
    hipStream_t s = (hipStream_t)stream;
    if ((st = register_batch_impl(b, b->ident, b->mask, b->alt, s)) != UPS_OK) return st;
    return launch_fallback_merge(b->n, results_d, b->alt, b->mask, s);
}

ups_status ups_register_batch_fallback(ups_context *ctx, ups_batch *b, double min_inlier_ratio,
                                       ups_icp_result *results_d, void *stream) {
    ups_status st = ups_batch_fallback_plan(ctx, b, min_inlier_ratio, results_d, nullptr, stream);
    if (st != UPS_OK) return st;
    return ups_batch_fallback_run(ctx, b, results_d, stream);
}

}  // extern "C"
