// Kernels of the pose-proposal network (BF16 MFMA convolutions, FP32 head,
// loss and Adam) and the launchers the proposal object and the layer-level
// C entry points share.
#pragma once

#include <algorithm>
#include <cmath>

#include "ups_internal.hpp"

namespace ups {

constexpr int kCnnOut = 6;  // (omega, t) of the proposed pose

// A 3x3 convolution on NHWC tensors: width circular, height zero-padded,
// output (h-1)/stride+1 x (w-1)/stride+1.
struct ConvShape {
    int n, h, w, cin, cout, stride, ho, wo;
};

ConvShape conv_shape(int n, int h, int w, int cin, int cout, int stride);
ups_status conv_check(const ConvShape &c);
int64_t conv_wgt_work_floats(const ConvShape &c);
ups_status launch_conv_fwd(const ConvShape &c, const uint16_t *x, const uint16_t *w_nk, const float *b, uint16_t *y,
                           hipStream_t s);
ups_status launch_conv_bwd_data(const ConvShape &c, const uint16_t *y, const float *dy, const uint16_t *w_kn,
                                float *dx, hipStream_t s);
ups_status launch_conv_bwd_weight(const ConvShape &c, const uint16_t *x, const uint16_t *y, const float *dy,
                                  float *dw, float *db, float *work, int64_t work_floats, hipStream_t s);
ups_status launch_fc_fwd(int n, int feat, const uint16_t *f, const float *Wfc, const float *bfc, float *out,
                         hipStream_t s);
ups_status launch_loss(int n, const float *y, const float *target, float *dout, float *loss, hipStream_t s);
ups_status launch_fc_bwd(int n, int feat, const uint16_t *f, const float *dout, const float *Wfc, float *dWfc,
                         float *dbfc, float *df, hipStream_t s);
ups_status launch_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, int64_t step,
                       hipStream_t s);
ups_status launch_pack_weight(int K, int N, const float *W, uint16_t *w_kn, uint16_t *w_nk, hipStream_t s);

}  // namespace ups
