// Convolution, fully connected, loss and Adam kernels of the pose-proposal
// network (BF16 operands on the matrix cores, FP32 accumulation).
//
// Every convolution pass is an implicit GEMM on one tile engine: a 256-thread
// block computes a 64 x 64 tile of C = A B, staging 64 x KB slices of A and B
// through LDS as bfloat16 and issuing gfx950's v_mfma_f32_16x16x32_bf16 (each
// wavefront owns a 32 x 32 quarter: 2 x 2 MFMA tiles, 32 k per instruction;
// v_mfma_f32_16x16x16_bf16 when K is at most 32 and the slice is 16 wide).
// The K loop loads the next slice into registers while the matrix cores work
// on the current one.  Operand loaders gather A and B
// straight from the NHWC activations, so no im2col buffer exists:
//   forward          C[pixel_out][cout] = X_col[pixel_out][(tap,ci)] W[(tap,ci)][cout]
//   backward (data)  C[pixel_in][ci]    = G_col[pixel_in][(tap,co)]  W[(tap,ci)][co]^T
//   backward (wgt)   C[(tap,ci)|1][co]  = X_col^T[(tap,ci)|1][pixel] G[pixel][co]   (split over pixels)
// with G = dL/dy masked by y > 0 (ReLU), taps (ky, kx) of a 3x3 window, the
// width circular and the height zero-padded.
#include <cstdint>

#include "ups_cnn.hpp"

namespace ups {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// round to nearest even
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int kBM = 64, kBN = 64;
constexpr int kSplitAlign = 16;                              // weight-gradient pixel chunks: multiples of this

// One 64 x 64 tile: A rows m0.., B columns n0.., K range [k_begin, k_end).
// LA::load(row, k, out[4]) / LB::load(col, k, out[4]) return bf16 values of
// A(row, k..k+3) / B(k..k+3, col), zero outside the operand; ST::store(row,
// col, v) writes one result.
template <int KB = 32, class LA, class LB, class ST>
__device__ __forceinline__ void mfma_tile(const LA &la, const LB &lb, const ST &st, int m0, int n0, int M, int N,
                                          int k_begin, int k_end) {
    // 32-wide k chunks on the 16x16x32 instruction when the slice holds them
    constexpr bool kX32 = KB % 32 == 0;
    // LDS row pitch (elements), padded to spread the rows over the banks and
    // keeping each row 16-byte aligned for the 8-element fragment loads
    constexpr int kLP = kX32 ? KB + 8 : KB + 4;
    constexpr int kQ = KB / 16;  // k quads per thread and operand in one slice
    __shared__ __align__(16) uint16_t As[kBM * kLP];
    __shared__ __align__(16) uint16_t Bs[kBN * kLP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = tid >> 2, lq = tid & 3;  // loader: row / column lr of the tile, k quads lq + 4 q
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    uint16_t a[kQ][4], b[kQ][4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int q = 0; q < kQ; q++) {
            const int k = k0 + 4 * (lq + 4 * q);
            la.load(m0 + lr, k, k_end, a[q]);
            lb.load(n0 + lr, k, k_end, b[q]);
        }
    };
    if (k_begin < k_end) fetch(k_begin);
    for (int k0 = k_begin; k0 < k_end; k0 += KB) {
#pragma unroll
        for (int q = 0; q < kQ; q++) {
            const int o = lr * kLP + 4 * (lq + 4 * q);
            *(uint2 *)&As[o] = make_uint2(a[q][0] | ((uint32_t)a[q][1] << 16), a[q][2] | ((uint32_t)a[q][3] << 16));
            *(uint2 *)&Bs[o] = make_uint2(b[q][0] | ((uint32_t)b[q][1] << 16), b[q][2] | ((uint32_t)b[q][3] << 16));
        }
        __syncthreads();
        // the next slice's loads are in flight while this slice is multiplied
        if (k0 + KB < k_end) fetch(k0 + KB);
        // chunks of the slice in ascending k.  Lane l carries row (A) or
        // column (B) l % 16 and the chunk's k = w (l / 16) .. w (l / 16) + w-1
        // (w = 8 or 4 elements): the same k in the same slot of both operands
        if constexpr (kX32) {
#pragma unroll
            for (int kc = 0; kc < KB / 32; kc++) {
                bf16x8 fa[2], fb[2];
#pragma unroll
                for (int i = 0; i < 2; i++)
                    fa[i] = *(const bf16x8 *)&As[(32 * wm + 16 * i + (lane & 15)) * kLP + 32 * kc + 8 * (lane >> 4)];
#pragma unroll
                for (int j = 0; j < 2; j++)
                    fb[j] = *(const bf16x8 *)&Bs[(32 * wn + 16 * j + (lane & 15)) * kLP + 32 * kc + 8 * (lane >> 4)];
#pragma unroll
                for (int i = 0; i < 2; i++)
#pragma unroll
                    for (int j = 0; j < 2; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kc = 0; kc < kQ; kc++) {
                bf16x4 fa[2], fb[2];
#pragma unroll
                for (int i = 0; i < 2; i++)
                    fa[i] = *(const bf16x4 *)&As[(32 * wm + 16 * i + (lane & 15)) * kLP + 16 * kc + 4 * (lane >> 4)];
#pragma unroll
                for (int j = 0; j < 2; j++)
                    fb[j] = *(const bf16x4 *)&Bs[(32 * wn + 16 * j + (lane & 15)) * kLP + 16 * kc + 4 * (lane >> 4)];
#pragma unroll
                for (int i = 0; i < 2; i++)
#pragma unroll
                    for (int j = 0; j < 2; j++)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[i], fb[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // D[4 (lane/16) + e][lane % 16] of each 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = m0 + 32 * wm + 16 * i + 4 * (lane >> 4) + e;
                const int col = n0 + 32 * wn + 16 * j + (lane & 15);
                if (row < M && col < N) st.store(row, col, acc[i][j][e]);
            }
}

// ------------------------------------------------------------ forward

// A = the 3x3 windows of the input: row = output pixel (b, oy, ox), column
// k = tap * cin + ci with tap = 3 ky + kx.
struct LoadIm2col {
    ConvShape c;
    const uint16_t *x;
    float inv_cin;  // 1 / cin
    // k / cin without an integer division: (k + 1/2) / cin lies at least
    // 1 / (2 cin) away from an integer, and the FP32 product (below 9, as
    // k < 9 cin) is within 9 * 2^-22 of it, so the truncation is exact for
    // any cin below 2^17
    __device__ __forceinline__ int tap_of(int k) const { return (int)(((float)k + 0.5f) * inv_cin); }
    __device__ __forceinline__ uint16_t at(int b, int oy, int ox, int k) const {
        const int tap = tap_of(k), ci = k - tap * c.cin;
        const int ky = tap / 3, kx = tap - 3 * ky;
        const int iy = c.stride * oy + ky - 1;
        if (iy < 0 || iy >= c.h) return 0;
        int ix = c.stride * ox + kx - 1;
        ix = ix < 0 ? ix + c.w : (ix >= c.w ? ix - c.w : ix);
        return x[((size_t)(b * c.h + iy) * c.w + ix) * c.cin + ci];
    }
    __device__ __forceinline__ void load(int m, int k, int k_end, uint16_t *o) const {
        const int P = c.n * c.ho * c.wo;
        if (m >= P) {
            o[0] = o[1] = o[2] = o[3] = 0;
            return;
        }
        const int b = m / (c.ho * c.wo), r = m - b * c.ho * c.wo, oy = r / c.wo, ox = r - oy * c.wo;
        if ((c.cin & 3) == 0 && k + 3 < k_end) {
            // four channels of one tap: one 8-byte load
            const int tap = tap_of(k), ci = k - tap * c.cin;
            const int ky = tap / 3, kx = tap - 3 * ky;
            const int iy = c.stride * oy + ky - 1;
            if (iy < 0 || iy >= c.h) {
                o[0] = o[1] = o[2] = o[3] = 0;
                return;
            }
            int ix = c.stride * ox + kx - 1;
            ix = ix < 0 ? ix + c.w : (ix >= c.w ? ix - c.w : ix);
            const uint2 v = *(const uint2 *)&x[((size_t)(b * c.h + iy) * c.w + ix) * c.cin + ci];
            o[0] = v.x & 0xFFFF, o[1] = v.x >> 16, o[2] = v.y & 0xFFFF, o[3] = v.y >> 16;
            return;
        }
        if ((c.cin & 1) == 0 && k + 3 < k_end) {
            // even cin (k is a multiple of 4): two channel pairs, each of one tap
#pragma unroll
            for (int p = 0; p < 2; p++) {
                const int kk = k + 2 * p, tap = tap_of(kk), ci = kk - tap * c.cin;
                const int ky = tap / 3, kx = tap - 3 * ky;
                const int iy = c.stride * oy + ky - 1;
                uint32_t v = 0;
                if (iy >= 0 && iy < c.h) {
                    int ix = c.stride * ox + kx - 1;
                    ix = ix < 0 ? ix + c.w : (ix >= c.w ? ix - c.w : ix);
                    v = *(const uint32_t *)&x[((size_t)(b * c.h + iy) * c.w + ix) * c.cin + ci];
                }
                o[2 * p] = v & 0xFFFF, o[2 * p + 1] = v >> 16;
            }
            return;
        }
#pragma unroll
        for (int e = 0; e < 4; e++) o[e] = (k + e < k_end) ? at(b, oy, ox, k + e) : 0;
    }
};

// B^T rows: W^T[cout][K] (bf16, K contiguous).
struct LoadRowsBf16 {
    const uint16_t *w;
    int rows, K;
    __device__ __forceinline__ void load(int n, int k, int k_end, uint16_t *o) const {
        if (n >= rows) {
            o[0] = o[1] = o[2] = o[3] = 0;
            return;
        }
        const uint16_t *p = w + (size_t)n * K;
        if ((K & 3) == 0 && k + 3 < k_end) {
            // rows start on 8-byte boundaries: one 8-byte load
            const uint2 v = *(const uint2 *)&p[k];
            o[0] = v.x & 0xFFFF, o[1] = v.x >> 16, o[2] = v.y & 0xFFFF, o[3] = v.y >> 16;
            return;
        }
#pragma unroll
        for (int e = 0; e < 4; e++) o[e] = (k + e < k_end) ? p[k + e] : 0;
    }
};

struct StoreReluBf16 {
    const float *bias;
    uint16_t *y;
    int N;
    __device__ __forceinline__ void store(int m, int n, float v) const {
        y[(size_t)m * N + n] = f2bf(fmaxf(v + bias[n], 0.f));
    }
};

template <int KB>
__global__ __launch_bounds__(256) void k_conv_fwd(ConvShape c, const uint16_t *__restrict__ x,
                                                  const uint16_t *__restrict__ w_nk, const float *__restrict__ bias,
                                                  uint16_t *__restrict__ y) {
    const int M = c.n * c.ho * c.wo, N = c.cout, K = 9 * c.cin;
    mfma_tile<KB>(LoadIm2col{c, x, 1.f / (float)c.cin}, LoadRowsBf16{w_nk, N, K}, StoreReluBf16{bias, y, N}, blockIdx.x * kBM,
              blockIdx.y * kBN, M, N, 0, K);
}

// ------------------------------------------------------ backward (data)

// g = dy masked by y > 0, rounded to bf16
__device__ __forceinline__ uint16_t grad_bf(const float *dy, const uint16_t *y, size_t idx) {
    return (y[idx] != 0 && !(y[idx] & 0x8000)) ? f2bf(dy[idx]) : (uint16_t)0;
}

// A row = input pixel (b, iy, ix), column k = tap * cout + co: the output
// gradient at the output pixel whose tap (ky, kx) reads (iy, ix), if any.
struct LoadGradCol {
    ConvShape c;
    const float *dy;
    const uint16_t *y;
    float inv_cout;  // 1 / cout: k / cout as in LoadIm2col::tap_of
    __device__ __forceinline__ void load(int m, int k, int k_end, uint16_t *o) const {
        o[0] = o[1] = o[2] = o[3] = 0;
        if (m >= c.n * c.h * c.w || k >= k_end) return;
        const int b = m / (c.h * c.w), r = m - b * c.h * c.w, iy = r / c.w, ix = r - iy * c.w;
        // cout is a multiple of 4: the four columns share a tap
        const int tap = (int)(((float)k + 0.5f) * inv_cout), co = k - tap * c.cout;
        const int ky = tap / 3, kx = tap - 3 * ky;
        const int sh = c.stride >> 1;  // stride 1 or 2
        const int ty = iy + 1 - ky;
        if (ty < 0 || (ty & sh) != 0 || (ty >> sh) >= c.ho) return;
        int tx = ix + 1 - kx;
        tx = tx < 0 ? tx + c.w : (tx >= c.w ? tx - c.w : tx);
        if ((tx & sh) != 0 || (tx >> sh) >= c.wo) return;
        const size_t base = ((size_t)(b * c.ho + (ty >> sh)) * c.wo + (tx >> sh)) * c.cout + co;
        // four consecutive channels: one 8-byte load of y, one 16-byte load of dy
        const uint2 yv = *(const uint2 *)&y[base];
        const float4 g = *(const float4 *)&dy[base];
        const uint16_t yy[4] = {(uint16_t)(yv.x & 0xFFFF), (uint16_t)(yv.x >> 16), (uint16_t)(yv.y & 0xFFFF),
                                (uint16_t)(yv.y >> 16)};
        const float gg[4] = {g.x, g.y, g.z, g.w};
#pragma unroll
        for (int e = 0; e < 4; e++) o[e] = (yy[e] != 0 && !(yy[e] & 0x8000)) ? f2bf(gg[e]) : (uint16_t)0;
    }
};

// B^T row n = ci: W[(tap, ci)][co] over k = tap * cout + co (4 co contiguous).
struct LoadWkn {
    ConvShape c;
    const uint16_t *w_kn;
    float inv_cout;
    __device__ __forceinline__ void load(int n, int k, int k_end, uint16_t *o) const {
        o[0] = o[1] = o[2] = o[3] = 0;
        if (n >= c.cin || k >= k_end) return;
        const int tap = (int)(((float)k + 0.5f) * inv_cout), co = k - tap * c.cout;
        const uint2 v = *(const uint2 *)&w_kn[((size_t)tap * c.cin + n) * c.cout + co];
        o[0] = v.x & 0xFFFF, o[1] = v.x >> 16, o[2] = v.y & 0xFFFF, o[3] = v.y >> 16;
    }
};

struct StoreF32 {
    float *out;
    int N;
    __device__ __forceinline__ void store(int m, int n, float v) const { out[(size_t)m * N + n] = v; }
};

__global__ __launch_bounds__(256) void k_conv_bwd_data(ConvShape c, const uint16_t *__restrict__ y,
                                                       const float *__restrict__ dy,
                                                       const uint16_t *__restrict__ w_kn, float *__restrict__ dx) {
    const int M = c.n * c.h * c.w, N = c.cin, K = 9 * c.cout;
    const float inv_cout = 1.f / (float)c.cout;
    mfma_tile(LoadGradCol{c, dy, y, inv_cout}, LoadWkn{c, w_kn, inv_cout}, StoreF32{dx, N}, blockIdx.x * kBM,
              blockIdx.y * kBN, M, N, 0, K);
}

// ---------------------------------------------------- backward (weights)

// A row r = (tap, ci) for r < 9 cin, the bias row (all ones) for r = 9 cin;
// column k = output pixel.
struct LoadIm2colT {
    ConvShape c;
    const uint16_t *x;
    __device__ __forceinline__ void load(int r, int k, int k_end, uint16_t *o) const {
        const int K9 = 9 * c.cin;
        o[0] = o[1] = o[2] = o[3] = 0;
        if (r > K9 || k >= k_end) return;
        if (r == K9) {
#pragma unroll
            for (int e = 0; e < 4; e++) o[e] = (k + e < k_end) ? (uint16_t)0x3F80 : (uint16_t)0;  // 1.0
            return;
        }
        const int tap = r / c.cin, ci = r - tap * c.cin;
        const int ky = tap / 3, kx = tap - 3 * ky;
        // the first pixel's (b, oy, ox) by division, the next three by stepping
        int b = k / (c.ho * c.wo), q = k - b * c.ho * c.wo, oy = q / c.wo, ox = q - oy * c.wo;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            if (k + e < k_end) {
                const int iy = c.stride * oy + ky - 1;
                if (iy >= 0 && iy < c.h) {
                    int ix = c.stride * ox + kx - 1;
                    ix = ix < 0 ? ix + c.w : (ix >= c.w ? ix - c.w : ix);
                    o[e] = x[((size_t)(b * c.h + iy) * c.w + ix) * c.cin + ci];
                }
            }
            if (++ox == c.wo) {
                ox = 0;
                if (++oy == c.ho) {
                    oy = 0;
                    b++;
                }
            }
        }
    }
};

// B^T row n = co over k = output pixel: G[pixel][co].
struct LoadGradT {
    ConvShape c;
    const float *dy;
    const uint16_t *y;
    __device__ __forceinline__ void load(int n, int k, int k_end, uint16_t *o) const {
#pragma unroll
        for (int e = 0; e < 4; e++)
            o[e] = (n < c.cout && k + e < k_end) ? grad_bf(dy, y, (size_t)(k + e) * c.cout + n) : (uint16_t)0;
    }
};

// blockIdx.z = split s over output pixels [s chunk, (s+1) chunk)
__global__ __launch_bounds__(256) void k_conv_bwd_weight(ConvShape c, const uint16_t *__restrict__ x,
                                                         const uint16_t *__restrict__ y, const float *__restrict__ dy,
                                                         int chunk, float *__restrict__ part) {
    const int M = 9 * c.cin + 1, N = c.cout, P = c.n * c.ho * c.wo;
    const int kb = blockIdx.z * chunk, ke = min(P, kb + chunk);
    mfma_tile(LoadIm2colT{c, x}, LoadGradT{c, dy, y}, StoreF32{part + (size_t)blockIdx.z * M * N, N},
              blockIdx.x * kBM, blockIdx.y * kBN, M, N, kb, ke);
}

// dW[r][co] (r < 9 cin) and db[co] (the ones row): sum of the splits in order.
__global__ __launch_bounds__(256) void k_conv_bwd_weight_reduce(int M, int N, int splits,
                                                                const float *__restrict__ part, float *__restrict__ dw,
                                                                float *__restrict__ db) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= M * N) return;
    float s = 0.f;
    for (int z = 0; z < splits; z++) s += part[(size_t)z * M * N + i];
    const int r = i / N;
    if (r < M - 1) dw[i] = s;
    else db[i - r * N] = s;
}

// The same sums for few outputs and many splits (the first layers): one
// wavefront per output, lane l adding splits l, l + 64, ... in order, then a
// xor butterfly over the lanes (every lane ends with the same total).
__global__ __launch_bounds__(256) void k_conv_bwd_weight_reduce_wave(int M, int N, int splits,
                                                                     const float *__restrict__ part,
                                                                     float *__restrict__ dw, float *__restrict__ db) {
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= M * N) return;  // uniform per wavefront
    float s = 0.f;
    for (int z = lane; z < splits; z += 64) s += part[(size_t)z * M * N + i];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
    if (lane != 0) return;
    const int r = i / N;
    if (r < M - 1) dw[i] = s;
    else db[i - r * N] = s;
}

// ------------------------------------------------------------ host side

static int cdiv(int a, int b) { return (a + b - 1) / b; }

ConvShape conv_shape(int n, int h, int w, int cin, int cout, int stride) {
    ConvShape c;
    c.n = n, c.h = h, c.w = w, c.cin = cin, c.cout = cout, c.stride = stride;
    c.ho = (h - 1) / stride + 1;
    c.wo = (w - 1) / stride + 1;
    return c;
}

ups_status conv_check(const ConvShape &c) {
    UPS_REQUIRE(c.n >= 0 && c.h >= 1 && c.w >= 2 && c.cin >= 1 && c.cin <= 65536 && c.cout >= 4 &&
                    c.cout <= 65536 && (c.cout & 3) == 0,
                "conv shape: need n >= 0, h >= 1, w >= 2, 1 <= cin <= 65536, cout a multiple of 4 in [4, 65536]");
    UPS_REQUIRE(c.stride == 1 || c.stride == 2, "conv stride must be 1 or 2");
    UPS_REQUIRE(c.w % c.stride == 0, "conv width must be a multiple of the stride");
    UPS_REQUIRE((int64_t)c.n * c.h * c.w * (c.cin > c.cout ? c.cin : c.cout) < ((int64_t)1 << 31),
                "conv tensors too large");
    return UPS_OK;
}

ups_status launch_conv_fwd(const ConvShape &c, const uint16_t *x, const uint16_t *w_nk, const float *b, uint16_t *y,
                           hipStream_t s) {
    const int M = c.n * c.ho * c.wo;
    if (M == 0) return UPS_OK;
    // a small K (the first layer's 9 x 2 = 18) wastes less in 16-wide slices
    if (9 * c.cin <= 32)
        hipLaunchKernelGGL(k_conv_fwd<16>, dim3(cdiv(M, kBM), cdiv(c.cout, kBN)), dim3(256), 0, s, c, x, w_nk, b, y);
    else
        hipLaunchKernelGGL(k_conv_fwd<32>, dim3(cdiv(M, kBM), cdiv(c.cout, kBN)), dim3(256), 0, s, c, x, w_nk, b, y);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_conv_bwd_data(const ConvShape &c, const uint16_t *y, const float *dy, const uint16_t *w_kn,
                                float *dx, hipStream_t s) {
    const int M = c.n * c.h * c.w;
    if (M == 0) return UPS_OK;
    hipLaunchKernelGGL(k_conv_bwd_data, dim3(cdiv(M, kBM), cdiv(c.cin, kBN)), dim3(256), 0, s, c, y, dy, w_kn, dx);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

// Splits of the output pixels for the weight gradient: about 1024 blocks,
// chunks a multiple of kSplitAlign and at least 64 pixels.
static void wgt_split(const ConvShape &c, int &splits, int &chunk) {
    const int M = 9 * c.cin + 1, P = c.n * c.ho * c.wo;
    const int tiles = cdiv(M, kBM) * cdiv(c.cout, kBN);
    splits = std::max(1, std::min(256, cdiv(1024, tiles)));
    chunk = std::max(64, cdiv(cdiv(std::max(P, 1), splits), kSplitAlign) * kSplitAlign);
    splits = cdiv(std::max(P, 1), chunk);
}

int64_t conv_wgt_work_floats(const ConvShape &c) {
    int splits, chunk;
    wgt_split(c, splits, chunk);
    return (int64_t)splits * (9 * c.cin + 1) * c.cout;
}

ups_status launch_conv_bwd_weight(const ConvShape &c, const uint16_t *x, const uint16_t *y, const float *dy,
                                  float *dw, float *db, float *work, int64_t work_floats, hipStream_t s) {
    int splits, chunk;
    wgt_split(c, splits, chunk);
    const int M = 9 * c.cin + 1;
    UPS_REQUIRE((int64_t)splits * M * c.cout <= work_floats, "weight-gradient workspace too small");
    const int P = c.n * c.ho * c.wo;
    if (P > 0) {
        hipLaunchKernelGGL(k_conv_bwd_weight, dim3(cdiv(M, kBM), cdiv(c.cout, kBN), splits), dim3(256), 0, s, c, x, y,
                           dy, chunk, work);
        UPS_CHECK_HIP(hipGetLastError());
    }
    if (M * c.cout <= 32768 && splits >= 64)
        hipLaunchKernelGGL(k_conv_bwd_weight_reduce_wave, dim3(cdiv(M * c.cout, 4)), dim3(256), 0, s, M, c.cout,
                           P > 0 ? splits : 0, work, dw, db);
    else
        hipLaunchKernelGGL(k_conv_bwd_weight_reduce, dim3(cdiv(M * c.cout, 256)), dim3(256), 0, s, M, c.cout,
                           P > 0 ? splits : 0, work, dw, db);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

// ------------------------------------------------- head, loss, optimiser

// y[b][o] = bfc[o] + sum_k f[b][k] Wfc[o][k]; one block per sample, fixed-order sums.
__global__ __launch_bounds__(256) void k_fc_fwd(int feat, const uint16_t *__restrict__ f, const float *__restrict__ Wfc,
                                                const float *__restrict__ bfc, float *__restrict__ out) {
    __shared__ float red[kCnnOut][256];
    const int b = blockIdx.x, t = threadIdx.x;
    float s[kCnnOut] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = t; k < feat; k += 256) {
        const float v = bf2f(f[(size_t)b * feat + k]);
#pragma unroll
        for (int o = 0; o < kCnnOut; o++) s[o] = fmaf(v, Wfc[(size_t)o * feat + k], s[o]);
    }
#pragma unroll
    for (int o = 0; o < kCnnOut; o++) red[o][t] = s[o];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int o = 0; o < kCnnOut; o++) red[o][t] += red[o][t + w];
        __syncthreads();
    }
    if (t < kCnnOut) out[b * kCnnOut + t] = red[t][0] + bfc[t];
}

// dout = (y - target) / n and loss = sum (y - target)^2 / (2 n); one block.
__global__ __launch_bounds__(256) void k_loss(int n, const float *__restrict__ y, const float *__restrict__ target,
                                              float *__restrict__ dout, float *__restrict__ loss) {
    __shared__ float red[256];
    const int t = threadIdx.x;
    const float inv = 1.f / (float)n;
    float s = 0.f;
    for (int i = t; i < n * kCnnOut; i += 256) {
        const float d = y[i] - target[i];
        dout[i] = d * inv;
        s = fmaf(d, d, s);
    }
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0 && loss) *loss = red[0] * 0.5f * inv;
}

// dWfc[o][k] = sum_b dout[b][o] f[b][k], dbfc[o] = sum_b dout[b][o] (samples in order)
__global__ __launch_bounds__(256) void k_fc_bwd_w(int n, int feat, const uint16_t *__restrict__ f,
                                                  const float *__restrict__ dout, float *__restrict__ dWfc,
                                                  float *__restrict__ dbfc) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k < feat) {
        float s[kCnnOut] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int b = 0; b < n; b++) {
            const float v = bf2f(f[(size_t)b * feat + k]);
#pragma unroll
            for (int o = 0; o < kCnnOut; o++) s[o] = fmaf(dout[b * kCnnOut + o], v, s[o]);
        }
#pragma unroll
        for (int o = 0; o < kCnnOut; o++) dWfc[(size_t)o * feat + k] = s[o];
    }
    if (blockIdx.x == 0 && threadIdx.x < kCnnOut) {
        float s = 0.f;
        for (int b = 0; b < n; b++) s += dout[b * kCnnOut + threadIdx.x];
        dbfc[threadIdx.x] = s;
    }
}

// df[b][k] = sum_o dout[b][o] Wfc[o][k]
__global__ __launch_bounds__(256) void k_fc_bwd_x(int n, int feat, const float *__restrict__ dout,
                                                  const float *__restrict__ Wfc, float *__restrict__ df) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n * feat) return;
    const int b = i / feat, k = i - b * feat;
    float s = 0.f;
#pragma unroll
    for (int o = 0; o < kCnnOut; o++) s = fmaf(dout[b * kCnnOut + o], Wfc[(size_t)o * feat + k], s);
    df[i] = s;
}

// Adam (Kingma and Ba): c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ __launch_bounds__(256) void k_adam(int64_t n, float *__restrict__ p, const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v, float lr, float beta1,
                                              float beta2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// bf16 copies of a conv weight W[K][N] (FP32): w_kn = W, w_nk = W^T
__global__ __launch_bounds__(256) void k_pack_weight(int K, int N, const float *__restrict__ W,
                                                     uint16_t *__restrict__ w_kn, uint16_t *__restrict__ w_nk) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= K * N) return;
    const int k = i / N, nn = i - k * N;
    const uint16_t h = f2bf(W[i]);
    w_kn[i] = h;
    w_nk[(size_t)nn * K + k] = h;
}

ups_status launch_fc_fwd(int n, int feat, const uint16_t *f, const float *Wfc, const float *bfc, float *out,
                         hipStream_t s) {
    if (n == 0) return UPS_OK;
    hipLaunchKernelGGL(k_fc_fwd, dim3(n), dim3(256), 0, s, feat, f, Wfc, bfc, out);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_loss(int n, const float *y, const float *target, float *dout, float *loss, hipStream_t s) {
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(256), 0, s, n, y, target, dout, loss);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_fc_bwd(int n, int feat, const uint16_t *f, const float *dout, const float *Wfc, float *dWfc,
                         float *dbfc, float *df, hipStream_t s) {
    hipLaunchKernelGGL(k_fc_bwd_w, dim3(cdiv(feat, 256)), dim3(256), 0, s, n, feat, f, dout, dWfc, dbfc);
    UPS_CHECK_HIP(hipGetLastError());
    if (n > 0) {
        hipLaunchKernelGGL(k_fc_bwd_x, dim3(cdiv(n * feat, 256)), dim3(256), 0, s, n, feat, dout, Wfc, df);
        UPS_CHECK_HIP(hipGetLastError());
    }
    return UPS_OK;
}

ups_status launch_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, int64_t step,
                       hipStream_t s) {
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)step)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)step)));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, p, g, m, v, lr, (float)b1,
                       (float)b2, 1e-8f, c1, c2);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_pack_weight(int K, int N, const float *W, uint16_t *w_kn, uint16_t *w_nk, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_weight, dim3(cdiv(K * N, 256)), dim3(256), 0, s, K, N, W, w_kn, w_nk);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
