// The pose-proposal network as a library object: parameters, Adam state,
// activations and workspace in device memory; forward, training step, input
// preparation from range images and conversion of the output to poses.  The
// network (five 3x3 BF16 convolutions with ReLU, then a 4096 -> 6 FP32 layer)
// proposes the scan -> keyframe pose that starts a registration; plain
// identity-started ICP remains the fallback (ups_register_batch_fallback).
#include <cstdio>
#include <cstring>
#include <vector>

#include "ups_cnn.hpp"

namespace ups {

namespace {

constexpr int kRows = UPS_PROPOSAL_ROWS, kCols = UPS_PROPOSAL_COLS, kIn = 2;
constexpr int kLayers = 5;
constexpr int kCin[kLayers] = {2, 32, 64, 96, 128};
constexpr int kCout[kLayers] = {32, 64, 96, 128, 128};
constexpr int kStride[kLayers] = {2, 2, 2, 2, 1};
constexpr double kSOmega = 0.25, kST = 1.0;  // output scales of omega (rad) and t (m)

struct Layout {
    int h[kLayers + 1], w[kLayers + 1];
    int64_t w_off[kLayers], b_off[kLayers], fcw_off, fcb_off, total;
    int64_t wb_off[kLayers], wb_total;  // bf16 weight copies
    int feat;
};

Layout make_layout() {
    Layout L;
    L.h[0] = kRows, L.w[0] = kCols;
    int64_t o = 0, ob = 0;
    for (int k = 0; k < kLayers; k++) {
        L.h[k + 1] = (L.h[k] - 1) / kStride[k] + 1;
        L.w[k + 1] = (L.w[k] - 1) / kStride[k] + 1;
        L.w_off[k] = o;
        o += 9 * kCin[k] * kCout[k];
        L.b_off[k] = o;
        o += kCout[k];
        L.wb_off[k] = ob;
        ob += 9 * kCin[k] * kCout[k];
    }
    L.feat = L.h[kLayers] * L.w[kLayers] * kCout[kLayers - 1];
    L.fcw_off = o;
    o += (int64_t)kCnnOut * L.feat;
    L.fcb_off = o;
    o += kCnnOut;
    L.total = o;
    L.wb_total = ob;
    return L;
}

const Layout &layout() {
    static const Layout L = make_layout();
    return L;
}


// One range image the input is taken from: range of pixel (i, j) at
// r[(i * cols + j) * stride].
struct RangeImg {
    const float *r;
    int rows, cols, stride;
    float r_min, r_max;
};

struct PropItem {
    RangeImg img[2];  // keyframe, scan
};

// x[b][y][x][c] = bf16(1/r) of pixel (y rows/32, x cols/256) of image c, 0
// where the range is not valid.
// A block covers 256 pixels of one pair, so the pair's descriptor is
// block-uniform (scalar loads); both images' ranges are loaded before
// either is used, and the two channels of a pixel go out as one 4-byte store.
__device__ __forceinline__ uint32_t prop_inv_range_bf16(const RangeImg &im, float r) {
    const bool ok = isfinite(r) && r > im.r_min && r <= im.r_max;
    const float v = ok ? 1.0f / r : 0.0f;
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

__global__ __launch_bounds__(256) void k_prop_input(const PropItem *__restrict__ items, int n, uint32_t *__restrict__ x) {
    static_assert((kRows * kCols) % 256 == 0, "a block covers pixels of one pair");
    static_assert(kIn == 2, "two channels per 4-byte store");
    constexpr int kBlocksPerPair = kRows * kCols / 256;
    const int b = blockIdx.x / kBlocksPerPair;
    if (b >= n) return;
    const int q = (blockIdx.x - b * kBlocksPerPair) * 256 + threadIdx.x, y = q / kCols, xx = q - y * kCols;
    const RangeImg &kf = items[b].img[0], &sc = items[b].img[1];
    const float r0 = kf.r[((size_t)(y * (kf.rows / kRows)) * kf.cols + (size_t)xx * (kf.cols / kCols)) * kf.stride];
    const float r1 = sc.r[((size_t)(y * (sc.rows / kRows)) * sc.cols + (size_t)xx * (sc.cols / kCols)) * sc.stride];
    x[(size_t)b * (kRows * kCols) + q] = prop_inv_range_bf16(kf, r0) | (prop_inv_range_bf16(sc, r1) << 16);
}

// pose[b] = (Exp(S_omega y[0:3]), S_t y[3:6]) in FP64 (Rodrigues).
__global__ void k_prop_pose(int n, const float *__restrict__ y, ups_pose *__restrict__ pose) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const double w0 = kSOmega * y[b * kCnnOut], w1 = kSOmega * y[b * kCnnOut + 1], w2 = kSOmega * y[b * kCnnOut + 2];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2, th = sqrt(th2);
    double A, B;
    if (th < 1e-8) {
        A = 1.0;
        B = 0.5;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
    }
    const double K[3][3] = {{0, -w2, w1}, {w2, 0, -w0}, {-w1, w0, 0}};
    ups_pose &P = pose[b];
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) {
            const double k2 = K[a][0] * K[0][c] + K[a][1] * K[1][c] + K[a][2] * K[2][c];
            P.R[3 * a + c] = (a == c ? 1.0 : 0.0) + A * K[a][c] + B * k2;
        }
    for (int a = 0; a < 3; a++) P.t[a] = kST * y[b * kCnnOut + 3 + a];
}

}  // namespace

}  // namespace ups

using namespace ups;

struct ups_proposal {
    int device = 0;
    int max_batch = 0;
    int64_t step = 0;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *w_kn = nullptr, *w_nk = nullptr;
    uint16_t *act = nullptr;  // input + five activations (bf16)
    float *dact = nullptr;    // gradients of the five activations
    int64_t act_off[kLayers + 1] = {}, dact_off[kLayers + 1] = {};
    float *out = nullptr, *dout = nullptr;
    float *work = nullptr;
    int64_t work_floats = 0;
    PropItem *d_items = nullptr;
    int n_items = 0;
};

namespace {

void free_prop(ups_proposal *p) {
    for (void *q : {(void *)p->params, (void *)p->grads, (void *)p->m, (void *)p->v, (void *)p->w_kn, (void *)p->w_nk,
                    (void *)p->act, (void *)p->dact, (void *)p->out, (void *)p->dout, (void *)p->work,
                    (void *)p->d_items})
        (void)hipFree(q);
    delete p;
}

ConvShape layer_shape(int k, int n) {
    const Layout &L = layout();
    return conv_shape(n, L.h[k], L.w[k], kCin[k], kCout[k], kStride[k]);
}

ups_status pack_all(ups_proposal *p, hipStream_t s) {
    const Layout &L = layout();
    for (int k = 0; k < kLayers; k++) {
        ups_status st = launch_pack_weight(9 * kCin[k], kCout[k], p->params + L.w_off[k], p->w_kn + L.wb_off[k],
                                           p->w_nk + L.wb_off[k], s);
        if (st != UPS_OK) return st;
    }
    return UPS_OK;
}

ups_status forward_impl(ups_proposal *p, int n, const uint16_t *x, float *y, hipStream_t s) {
    const Layout &L = layout();
    ups_status st;
    const uint16_t *in = x;
    for (int k = 0; k < kLayers; k++) {
        uint16_t *o = p->act + p->act_off[k + 1];
        if ((st = launch_conv_fwd(layer_shape(k, n), in, p->w_nk + L.wb_off[k], p->params + L.b_off[k], o, s)) !=
            UPS_OK)
            return st;
        in = o;
    }
    return launch_fc_fwd(n, L.feat, in, p->params + L.fcw_off, p->params + L.fcb_off, y, s);
}

ups_status check_n(const ups_proposal *p, int n) {
    UPS_REQUIRE(n >= 1 && n <= p->max_batch, "n must be in [1, the proposal's max_batch]");
    return UPS_OK;
}

}  // namespace

extern "C" {

int64_t ups_proposal_num_params(void) { return layout().total; }

ups_status ups_proposal_create(ups_context *ctx, int32_t max_batch, ups_proposal **out) {
    UPS_REQUIRE(ctx && out, "null argument");
    UPS_REQUIRE(max_batch >= 1 && max_batch <= 65536, "max_batch must be in [1, 65536]");
    *out = nullptr;
    DeviceGuard g(ctx->device);
    UPS_CHECK_HIP(g.err);
    const Layout &L = layout();
    ups_proposal *p = new ups_proposal();
    p->device = ctx->device;
    p->max_batch = max_batch;
    int64_t ao = 0, dofs = 0;
    p->act_off[0] = 0;
    ao = (int64_t)max_batch * kRows * kCols * kIn;
    for (int k = 0; k < kLayers; k++) {
        p->act_off[k + 1] = ao;
        p->dact_off[k + 1] = dofs;
        const int64_t sz = (int64_t)max_batch * L.h[k + 1] * L.w[k + 1] * kCout[k];
        ao += sz;
        dofs += sz;
        p->work_floats = std::max(p->work_floats, conv_wgt_work_floats(layer_shape(k, max_batch)));
    }
    hipError_t e = hipSuccess;
    auto alloc = [&](void **ptr, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(ptr, bytes);
    };
    alloc((void **)&p->params, L.total * sizeof(float));
    alloc((void **)&p->grads, L.total * sizeof(float));
    alloc((void **)&p->m, L.total * sizeof(float));
    alloc((void **)&p->v, L.total * sizeof(float));
    alloc((void **)&p->w_kn, L.wb_total * sizeof(uint16_t));
    alloc((void **)&p->w_nk, L.wb_total * sizeof(uint16_t));
    alloc((void **)&p->act, ao * sizeof(uint16_t));
    alloc((void **)&p->dact, dofs * sizeof(float));
    alloc((void **)&p->out, (size_t)max_batch * kCnnOut * sizeof(float));
    alloc((void **)&p->dout, (size_t)max_batch * kCnnOut * sizeof(float));
    alloc((void **)&p->work, p->work_floats * sizeof(float));
    alloc((void **)&p->d_items, (size_t)max_batch * sizeof(PropItem));
    if (e == hipSuccess) e = hipMemset(p->params, 0, L.total * sizeof(float));
    if (e == hipSuccess) e = hipMemset(p->grads, 0, L.total * sizeof(float));
    if (e == hipSuccess) e = hipMemset(p->m, 0, L.total * sizeof(float));
    if (e == hipSuccess) e = hipMemset(p->v, 0, L.total * sizeof(float));
    if (e == hipSuccess) e = hipMemset(p->w_kn, 0, L.wb_total * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemset(p->w_nk, 0, L.wb_total * sizeof(uint16_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_prop(p);
        set_error(std::string("proposal allocation failed: ") + hipGetErrorString(e));
        return UPS_ERR_HIP;
    }
    *out = p;
    return UPS_OK;
}

void ups_proposal_destroy(ups_proposal *p) {
    if (!p) return;
    DeviceGuard g(p->device);
    (void)hipDeviceSynchronize();
    free_prop(p);
}

ups_status ups_proposal_set_params(ups_proposal *p, const float *params_h, int64_t n) {
    UPS_REQUIRE(p && params_h, "null argument");
    UPS_REQUIRE(n == layout().total, "parameter count mismatch");
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    UPS_CHECK_HIP(hipMemcpy(p->params, params_h, n * sizeof(float), hipMemcpyHostToDevice));
    UPS_CHECK_HIP(hipMemset(p->m, 0, n * sizeof(float)));
    UPS_CHECK_HIP(hipMemset(p->v, 0, n * sizeof(float)));
    p->step = 0;
    ups_status st = pack_all(p, nullptr);
    if (st != UPS_OK) return st;
    UPS_CHECK_HIP(hipDeviceSynchronize());
    return UPS_OK;
}

ups_status ups_proposal_get_params(ups_proposal *p, float *params_h, int64_t n) {
    UPS_REQUIRE(p && params_h, "null argument");
    UPS_REQUIRE(n == layout().total, "parameter count mismatch");
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    UPS_CHECK_HIP(hipDeviceSynchronize());
    UPS_CHECK_HIP(hipMemcpy(params_h, p->params, n * sizeof(float), hipMemcpyDeviceToHost));
    return UPS_OK;
}

// Parameter file: the 8 bytes "UPSPRM01", the parameter count as a
// little-endian int64, then the FP32 parameters in the layout's order.
static const char kParamMagic[8] = {'U', 'P', 'S', 'P', 'R', 'M', '0', '1'};

ups_status ups_proposal_save(ups_proposal *p, const char *path) {
    UPS_REQUIRE(p && path, "null argument");
    const int64_t n = layout().total;
    std::vector<float> h(n);
    ups_status st = ups_proposal_get_params(p, h.data(), n);
    if (st != UPS_OK) return st;
    FILE *f = fopen(path, "wb");
    UPS_REQUIRE(f != nullptr, std::string("cannot open ") + path + " for writing");
    const bool ok = fwrite(kParamMagic, 1, 8, f) == 8 && fwrite(&n, sizeof(n), 1, f) == 1 &&
                    fwrite(h.data(), sizeof(float), n, f) == (size_t)n;
    const bool closed = fclose(f) == 0;
    UPS_REQUIRE(ok && closed, std::string("write to ") + path + " failed");
    return UPS_OK;
}

ups_status ups_proposal_load(ups_proposal *p, const char *path) {
    UPS_REQUIRE(p && path, "null argument");
    const int64_t n = layout().total;
    FILE *f = fopen(path, "rb");
    UPS_REQUIRE(f != nullptr, std::string("cannot open ") + path);
    char magic[8];
    int64_t m = -1;
    std::vector<float> h(n);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kParamMagic, 8) == 0 && fread(&m, sizeof(m), 1, f) == 1 &&
              m == n && fread(h.data(), sizeof(float), n, f) == (size_t)n;
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;  // nothing after the parameters
    fclose(f);
    UPS_REQUIRE(ok, std::string(path) + " is not a parameter file of this network");
    return ups_proposal_set_params(p, h.data(), n);
}

// Checkpoint file: the 8 bytes "UPSCKP01", the parameter count and the Adam
// step count as little-endian int64, then the FP32 parameters, first moments
// and second moments in the layout's order.
static const char kCkptMagic[8] = {'U', 'P', 'S', 'C', 'K', 'P', '0', '1'};

ups_status ups_proposal_save_checkpoint(ups_proposal *p, const char *path) {
    UPS_REQUIRE(p && path, "null argument");
    const int64_t n = layout().total;
    std::vector<float> h(3 * n);
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    UPS_CHECK_HIP(hipDeviceSynchronize());
    UPS_CHECK_HIP(hipMemcpy(h.data(), p->params, n * sizeof(float), hipMemcpyDeviceToHost));
    UPS_CHECK_HIP(hipMemcpy(h.data() + n, p->m, n * sizeof(float), hipMemcpyDeviceToHost));
    UPS_CHECK_HIP(hipMemcpy(h.data() + 2 * n, p->v, n * sizeof(float), hipMemcpyDeviceToHost));
    FILE *f = fopen(path, "wb");
    UPS_REQUIRE(f != nullptr, std::string("cannot open ") + path + " for writing");
    const int64_t step = p->step;
    const bool ok = fwrite(kCkptMagic, 1, 8, f) == 8 && fwrite(&n, sizeof(n), 1, f) == 1 &&
                    fwrite(&step, sizeof(step), 1, f) == 1 && fwrite(h.data(), sizeof(float), 3 * n, f) == (size_t)(3 * n);
    const bool closed = fclose(f) == 0;
    UPS_REQUIRE(ok && closed, std::string("write to ") + path + " failed");
    return UPS_OK;
}

ups_status ups_proposal_load_checkpoint(ups_proposal *p, const char *path) {
    UPS_REQUIRE(p && path, "null argument");
    const int64_t n = layout().total;
    FILE *f = fopen(path, "rb");
    UPS_REQUIRE(f != nullptr, std::string("cannot open ") + path);
    char magic[8];
    int64_t m = -1, step = -1;
    std::vector<float> h(3 * n);
    bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kCkptMagic, 8) == 0 && fread(&m, sizeof(m), 1, f) == 1 &&
              m == n && fread(&step, sizeof(step), 1, f) == 1 && step >= 0 &&
              fread(h.data(), sizeof(float), 3 * n, f) == (size_t)(3 * n);
    char extra;
    ok = ok && fread(&extra, 1, 1, f) == 0;
    fclose(f);
    UPS_REQUIRE(ok, std::string(path) + " is not a checkpoint of this network");
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    UPS_CHECK_HIP(hipDeviceSynchronize());
    UPS_CHECK_HIP(hipMemcpy(p->params, h.data(), n * sizeof(float), hipMemcpyHostToDevice));
    UPS_CHECK_HIP(hipMemcpy(p->m, h.data() + n, n * sizeof(float), hipMemcpyHostToDevice));
    UPS_CHECK_HIP(hipMemcpy(p->v, h.data() + 2 * n, n * sizeof(float), hipMemcpyHostToDevice));
    p->step = step;
    ups_status st = pack_all(p, nullptr);
    if (st != UPS_OK) return st;
    UPS_CHECK_HIP(hipDeviceSynchronize());
    return UPS_OK;
}

ups_status ups_proposal_activations(ups_proposal *p, int32_t layer, int32_t n, uint16_t *act_h, float *dact_h) {
    UPS_REQUIRE(p, "null argument");
    UPS_REQUIRE(layer >= 1 && layer <= kLayers, "layer must be in [1, 5]");
    ups_status st;
    if ((st = check_n(p, n)) != UPS_OK) return st;
    const Layout &L = layout();
    const size_t count = (size_t)n * L.h[layer] * L.w[layer] * kCout[layer - 1];
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    UPS_CHECK_HIP(hipDeviceSynchronize());
    if (act_h)
        UPS_CHECK_HIP(hipMemcpy(act_h, p->act + p->act_off[layer], count * sizeof(uint16_t), hipMemcpyDeviceToHost));
    if (dact_h)
        UPS_CHECK_HIP(hipMemcpy(dact_h, p->dact + p->dact_off[layer], count * sizeof(float), hipMemcpyDeviceToHost));
    return UPS_OK;
}

ups_status ups_proposal_get_grads(ups_proposal *p, float *grads_h, int64_t n) {
    UPS_REQUIRE(p && grads_h, "null argument");
    UPS_REQUIRE(n == layout().total, "parameter count mismatch");
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    UPS_CHECK_HIP(hipDeviceSynchronize());
    UPS_CHECK_HIP(hipMemcpy(grads_h, p->grads, n * sizeof(float), hipMemcpyDeviceToHost));
    return UPS_OK;
}

ups_status ups_proposal_plan_input(ups_proposal *p, int32_t n, const ups_range_image *kf_h,
                                   const ups_range_image *scan_h) {
    UPS_REQUIRE(p && kf_h && scan_h, "null argument");
    ups_status st;
    if ((st = check_n(p, n)) != UPS_OK) return st;
    std::vector<PropItem> items(n);
    for (int b = 0; b < n; b++) {
        for (int c = 0; c < 2; c++) {
            const ups_range_image &im = c == 0 ? kf_h[b] : scan_h[b];
            const std::string what = std::string(c == 0 ? "keyframe" : "scan") + " image " + std::to_string(b);
            UPS_REQUIRE(im.range_d != nullptr && ((uintptr_t)im.range_d % 4) == 0, what + ": null or misaligned");
            UPS_REQUIRE(im.rows >= kRows && im.cols >= kCols && im.rows % kRows == 0 && im.cols % kCols == 0,
                        what + ": rows / cols must be positive multiples of 32 / 256");
            UPS_REQUIRE(im.stride >= 1, what + ": stride must be >= 1");
            items[b].img[c] = RangeImg{im.range_d, im.rows, im.cols, im.stride, im.r_min, im.r_max};
        }
    }
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    UPS_CHECK_HIP(hipMemcpy(p->d_items, items.data(), n * sizeof(PropItem), hipMemcpyHostToDevice));
    p->n_items = n;
    return UPS_OK;
}

ups_status ups_proposal_input(ups_proposal *p, uint16_t *x_d, void *stream) {
    UPS_REQUIRE(p, "null argument");
    UPS_REQUIRE(p->n_items > 0, "no planned input (ups_proposal_plan_input)");
    ups_status st;
    uint16_t *x = x_d ? x_d : p->act;
    if ((st = check_ptr(x, 8, "input")) != UPS_OK) return st;
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    const int total = p->n_items * kRows * kCols;
    hipLaunchKernelGGL(k_prop_input, dim3((total + 255) / 256), dim3(256), 0, (hipStream_t)stream, p->d_items,
                       p->n_items, (uint32_t *)x);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status ups_proposal_forward(ups_proposal *p, int32_t n, const uint16_t *x_d, float *y_d, void *stream) {
    UPS_REQUIRE(p, "null argument");
    ups_status st;
    if ((st = check_n(p, n)) != UPS_OK) return st;
    const uint16_t *x = x_d ? x_d : p->act;
    if ((st = check_ptr(x, 8, "input")) != UPS_OK) return st;
    if ((st = check_ptr(y_d, 4, "output")) != UPS_OK) return st;
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    return forward_impl(p, n, x, y_d, (hipStream_t)stream);
}

ups_status ups_proposal_poses(ups_proposal *p, int32_t n, const float *y_d, ups_pose *poses_d, void *stream) {
    UPS_REQUIRE(p, "null argument");
    ups_status st;
    if ((st = check_n(p, n)) != UPS_OK) return st;
    if ((st = check_ptr(y_d, 4, "output")) != UPS_OK) return st;
    if ((st = check_ptr(poses_d, 8, "poses")) != UPS_OK) return st;
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    hipLaunchKernelGGL(k_prop_pose, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)stream, n, y_d, poses_d);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status ups_proposal_train_step(ups_proposal *p, int32_t n, const uint16_t *x_d, const float *target_d, float lr,
                                   float *loss_d, void *stream) {
    UPS_REQUIRE(p, "null argument");
    ups_status st;
    if ((st = check_n(p, n)) != UPS_OK) return st;
    const uint16_t *x = x_d ? x_d : p->act;
    if ((st = check_ptr(x, 8, "input")) != UPS_OK) return st;
    if ((st = check_ptr(target_d, 4, "target")) != UPS_OK) return st;
    UPS_REQUIRE(std::isfinite(lr) && lr >= 0.f, "lr must be finite and >= 0");
    DeviceGuard g(p->device);
    UPS_CHECK_HIP(g.err);
    hipStream_t s = (hipStream_t)stream;
    const Layout &L = layout();
    if ((st = forward_impl(p, n, x, p->out, s)) != UPS_OK) return st;
    if ((st = launch_loss(n, p->out, target_d, p->dout, loss_d, s)) != UPS_OK) return st;
    const uint16_t *feat = p->act + p->act_off[kLayers];
    if ((st = launch_fc_bwd(n, L.feat, feat, p->dout, p->params + L.fcw_off, p->grads + L.fcw_off,
                            p->grads + L.fcb_off, p->dact + p->dact_off[kLayers], s)) != UPS_OK)
        return st;
    for (int k = kLayers - 1; k >= 0; k--) {
        const ConvShape c = layer_shape(k, n);
        const uint16_t *in = k == 0 ? x : p->act + p->act_off[k];
        const uint16_t *y = p->act + p->act_off[k + 1];
        const float *dy = p->dact + p->dact_off[k + 1];
        if ((st = launch_conv_bwd_weight(c, in, y, dy, p->grads + L.w_off[k], p->grads + L.b_off[k], p->work,
                                         p->work_floats, s)) != UPS_OK)
            return st;
        if (k > 0 &&
            (st = launch_conv_bwd_data(c, y, dy, p->w_kn + L.wb_off[k], p->dact + p->dact_off[k], s)) != UPS_OK)
            return st;
    }
    p->step += 1;
    if ((st = launch_adam(L.total, p->params, p->grads, p->m, p->v, lr, p->step, s)) != UPS_OK) return st;
    return pack_all(p, s);
}

// ---- layer-level entry points

ups_status ups_conv3x3_forward(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t stride,
                               const uint16_t *x_d, const uint16_t *w_nk_d, const float *b_d, uint16_t *y_d,
                               void *stream) {
    const ConvShape c = conv_shape(n, h, w, cin, cout, stride);
    ups_status st;
    if ((st = conv_check(c)) != UPS_OK) return st;
    if (n == 0) return UPS_OK;
    if ((st = check_ptr(x_d, 8, "x")) != UPS_OK) return st;
    if ((st = check_ptr(w_nk_d, 8, "w")) != UPS_OK) return st;
    if ((st = check_ptr(b_d, 4, "b")) != UPS_OK) return st;
    if ((st = check_ptr(y_d, 2, "y")) != UPS_OK) return st;
    return launch_conv_fwd(c, x_d, w_nk_d, b_d, y_d, (hipStream_t)stream);
}

ups_status ups_conv3x3_backward_data(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t stride,
                                     const uint16_t *y_d, const float *dy_d, const uint16_t *w_kn_d, float *dx_d,
                                     void *stream) {
    const ConvShape c = conv_shape(n, h, w, cin, cout, stride);
    ups_status st;
    if ((st = conv_check(c)) != UPS_OK) return st;
    if (n == 0) return UPS_OK;
    if ((st = check_ptr(y_d, 8, "y")) != UPS_OK) return st;
    if ((st = check_ptr(dy_d, 16, "dy")) != UPS_OK) return st;
    if ((st = check_ptr(w_kn_d, 8, "w")) != UPS_OK) return st;
    if ((st = check_ptr(dx_d, 4, "dx")) != UPS_OK) return st;
    return launch_conv_bwd_data(c, y_d, dy_d, w_kn_d, dx_d, (hipStream_t)stream);
}

int64_t ups_conv3x3_backward_weight_work(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t stride) {
    const ConvShape c = conv_shape(n, h, w, cin, cout, stride);
    if (conv_check(c) != UPS_OK) return -1;
    return conv_wgt_work_floats(c);
}

ups_status ups_conv3x3_backward_weight(int32_t n, int32_t h, int32_t w, int32_t cin, int32_t cout, int32_t stride,
                                       const uint16_t *x_d, const uint16_t *y_d, const float *dy_d, float *dw_d,
                                       float *db_d, float *work_d, int64_t work_floats, void *stream) {
    const ConvShape c = conv_shape(n, h, w, cin, cout, stride);
    ups_status st;
    if ((st = conv_check(c)) != UPS_OK) return st;
    if ((st = check_ptr(dw_d, 4, "dw")) != UPS_OK) return st;
    if ((st = check_ptr(db_d, 4, "db")) != UPS_OK) return st;
    if ((st = check_ptr(work_d, 4, "work")) != UPS_OK) return st;
    if (n > 0) {
        if ((st = check_ptr(x_d, 8, "x")) != UPS_OK) return st;
        if ((st = check_ptr(y_d, 2, "y")) != UPS_OK) return st;
        if ((st = check_ptr(dy_d, 4, "dy")) != UPS_OK) return st;
    }
    return launch_conv_bwd_weight(c, x_d, y_d, dy_d, dw_d, db_d, work_d, work_floats, (hipStream_t)stream);
}

}  // extern "C"
