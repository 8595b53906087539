// Projective point-to-plane ICP (UPSLAM Section III-B, Equation 1) on gfx950.
//
// One launch = one Gauss-Newton iteration of one pyramid level:
//
//   0. every block reads the block partials left by the previous launch and
//      reduces them in the same fixed order, so every block solves the same
//      6x6 system (Cholesky, FP64) and applies the same update
//      T <- Exp(xi) T (FP64): no atomics, no fences, no extra solve launch --
//      the kernel boundary is the only synchronisation;
//   1. association of K pixels per thread at the new pose: rigid transform,
//      spherical re-projection into the keyframe, the Omega filter, the
//      point-to-plane residual r = (q - s1).n1 and J = [q x n1, n1];
//   2. the 29-value reduction [21 x J^T J | 6 x J^T r | r^2 | inliers]:
//      Kahan-compensated FP32 per thread, then FP64 (or plain FP32 in the
//      FP32 precision mode) DPP row sums and a fixed-order LDS sum per block,
//      written as one partial per block.
//
// The registration state (pose, status, flags) lives in two ping-pong slots:
// launch n reads slot n%2 and block 0 writes slot (n+1)%2.  Block partials are
// ping-ponged the same way.  A final evaluation launch applies the last update
// and accumulates the quality terms at level 0; a one-block finish launch
// writes the result.
//
// The same kernels serve one registration (descriptor passed by value) and a
// batch of registrations of different sizes (descriptors in device memory,
// block -> (registration, tile) through a per-level prefix table).
#include "ups_icp.hpp"

namespace ups {

// ---------------------------------------------------------------- reductions

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum over each 16-lane row (quad xor 1, quad xor 2, half-row mirror, row
// mirror); every lane of a row ends with the bitwise-same row sum.
template <typename T>
__device__ __forceinline__ T row_sum(T v) {
    if constexpr (sizeof(T) == 8) {
        v += dpp_d<0xB1>(v);
        v += dpp_d<0x4E>(v);
        v += dpp_d<0x141>(v);
        v += dpp_d<0x140>(v);
    } else {
        v += dpp_f<0xB1>(v);
        v += dpp_f<0x4E>(v);
        v += dpp_f<0x141>(v);
        v += dpp_f<0x140>(v);
    }
    return v;
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Sum NV per-thread values over the 256-thread block in a fixed order: DPP row
// sums, then the 16 row sums of each value added in row order.  tot[v] holds
// the block total of value v for every thread after the call.
template <int NV, typename Acc>
__device__ __forceinline__ void block_reduce(Acc (&x)[NV], Acc (*rows)[16], Acc *tot) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const Acc y = row_sum<Acc>(x[v]);
        if ((lane & 15) == 0) rows[v][wave * 4 + (lane >> 4)] = y;
    }
    __syncthreads();
    if (tid < NV) {
        Acc t = 0;
#pragma unroll
        for (int r = 0; r < 16; r++) t += rows[tid][r];
        tot[tid] = t;
    }
    __syncthreads();
}

// Load this thread's share of `n` block partials (partials t, t+256, ... for
// thread t) and add them up in that fixed order; block_reduce finishes.
template <int NV, typename Acc>
__device__ __forceinline__ void load_partials(const double *part, int n, Acc (&x)[NV]) {
#pragma unroll
    for (int v = 0; v < NV; v++) x[v] = 0;
    for (int b = threadIdx.x; b < n; b += kBlock) {
        const double *pb = part + (size_t)b * kPartialStride;
#pragma unroll
        for (int v = 0; v < NV; v++) x[v] += (Acc)pb[v];
    }
}

template <int NV, typename Acc>
__device__ __forceinline__ void reduce_partials(const double *part, int n, Acc (*rows)[16], Acc *tot) {
    Acc x[NV];
    load_partials<NV, Acc>(part, n, x);
    block_reduce<NV, Acc>(x, rows, tot);
}

// --------------------------------------------------------- FP64 / FP32 solve

template <typename T>
__device__ int cholesky_solve6(const T *A21, const T *b, T *xi) {
    T A[6][6], L[6][6], inv[6];
    int e = 0;
    for (int a = 0; a < 6; a++)
        for (int c = a; c < 6; c++) {
            A[a][c] = A21[e];
            A[c][a] = A21[e];
            e++;
        }
    T maxd = 0;
    for (int a = 0; a < 6; a++) maxd = A[a][a] > maxd ? A[a][a] : maxd;
    if (!(maxd > T(0))) return UPS_DEGENERATE;
    for (int c = 0; c < 6; c++) {
        T d = A[c][c];
        for (int k = 0; k < c; k++) d -= L[c][k] * L[c][k];
        if (!(d > T(1e-12) * maxd)) return UPS_DEGENERATE;
        L[c][c] = sqrt(d);
        inv[c] = T(1) / L[c][c];
        for (int r = c + 1; r < 6; r++) {
            T s = A[r][c];
            for (int k = 0; k < c; k++) s -= L[r][k] * L[c][k];
            L[r][c] = s * inv[c];
        }
    }
    T y[6];
    for (int r = 0; r < 6; r++) {
        T s = -b[r];
        for (int k = 0; k < r; k++) s -= L[r][k] * y[k];
        y[r] = s * inv[r];
    }
    for (int r = 5; r >= 0; r--) {
        T s = y[r];
        for (int k = r + 1; k < 6; k++) s -= L[k][r] * xi[k];
        xi[r] = s * inv[r];
    }
    return UPS_CONVERGED;
}

// R, t <- Exp(xi) (R, t) with xi = (omega, v): Rodrigues rotation and the V
// matrix.  Below |omega| = 1/4 the three coefficients sin(th)/th,
// (1-cos th)/th^2 and (th-sin th)/th^3 come from their Taylor series to the
// th^14 term (remainder < 1e-20), which avoids the cancellation of the closed
// forms and any sin/cos; above it the closed forms are used.
template <typename T>
__device__ void exp_compose(const T *xi, double *R, double *t) {
    const T w0 = xi[0], w1 = xi[1], w2 = xi[2];
    const T th2 = w0 * w0 + w1 * w1 + w2 * w2, th = sqrt(th2);
    T A, B, C;
    if (th < T(0.25)) {
        // 1/n! for n = 1..17
        constexpr double f[18] = {1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040,
                                  1.0 / 40320, 1.0 / 362880, 1.0 / 3628800, 1.0 / 39916800, 1.0 / 479001600,
                                  1.0 / 6227020800.0, 1.0 / 87178291200.0, 1.0 / 1307674368000.0,
                                  1.0 / 20922789888000.0, 1.0 / 355687428096000.0};
        A = B = C = 0;
        for (int k = 7; k >= 0; k--) {
            const T sg = (k & 1) ? T(-1) : T(1);
            A = A * th2 + sg * (T)f[2 * k + 1];
            B = B * th2 + sg * (T)f[2 * k + 2];
            C = C * th2 + sg * (T)f[2 * k + 3];
        }
    } else {
        A = sin(th) / th;
        B = (T(1) - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    const T K[3][3] = {{0, -w2, w1}, {w2, 0, -w0}, {-w1, w0, 0}};
    T K2[3][3], E[3][3], V[3][3];
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) K2[a][c] = K[a][0] * K[0][c] + K[a][1] * K[1][c] + K[a][2] * K[2][c];
    for (int a = 0; a < 3; a++)
        for (int c = 0; c < 3; c++) {
            const T I = (a == c) ? T(1) : T(0);
            E[a][c] = I + A * K[a][c] + B * K2[a][c];
            V[a][c] = I + B * K[a][c] + C * K2[a][c];
        }
    T te[3], Ro[9], to[3];
    for (int a = 0; a < 3; a++) te[a] = V[a][0] * xi[3] + V[a][1] * xi[4] + V[a][2] * xi[5];
    for (int k = 0; k < 9; k++) Ro[k] = (T)R[k];
    for (int k = 0; k < 3; k++) to[k] = (T)t[k];
    for (int a = 0; a < 3; a++) {
        for (int c = 0; c < 3; c++)
            R[3 * a + c] = (double)(E[a][0] * Ro[c] + E[a][1] * Ro[3 + c] + E[a][2] * Ro[6 + c]);
        t[a] = (double)(E[a][0] * to[0] + E[a][1] * to[1] + E[a][2] * to[2] + te[a]);
    }
}

// Gauss-Newton step from the reduced totals (thread 0).  Updates the state in
// place: pose, iteration count, step norm, convergence of the level, or the
// failure status that stops the registration with the pose unchanged.
template <typename T>
__device__ void gn_step(const StepArgs &a, const T *tot, RegState &S) {
    const double n_in = (double)tot[28];
    T xi[6];
    const int st = (n_in < (double)a.min_inliers) ? UPS_NO_INLIERS : cholesky_solve6<T>(tot, tot + 21, xi);
    if (st != UPS_CONVERGED) {
        S.status = st;
        S.stop = 1;
        return;
    }
    exp_compose<T>(xi, S.R, S.t);
    S.iters_run += 1;
    T nrm = 0;
    for (int k = 0; k < 6; k++) nrm += xi[k] * xi[k];
    S.last_norm = (double)sqrt(nrm);
    if (a.stop_norm > 0.0 && S.last_norm < a.stop_norm) S.level_active = 0;
}

// ------------------------------------------------------------------ kernel

// Partials a launch over `nblocks` blocks leaves for its successor: one per
// block, or a single folded one when there are more than 256.
__device__ __host__ __forceinline__ int npartials_of(int nblocks) { return nblocks > 256 ? 1 : nblocks; }

template <int K, int PREC, int MODE>
__device__ __forceinline__ void icp_block(const Inst &I, const StepArgs &a, int tile) {
    constexpr int NV = (MODE == MODE_ITER) ? 29 : 31;  // EVAL adds valid count and truncated cost
    using Acc = typename std::conditional<PREC == UPS_PREC_KAHAN_F64, double, float>::type;
    const int tid = threadIdx.x;
    const int l = a.level;
    const int ntiles = I.nblocks[l];
    RegState *slot_in = I.state + a.parity, *slot_out = I.state + (a.parity ^ 1);
    const double *part_in = I.partials + (size_t)a.parity * I.pstride * kPartialStride;
    double *part_out = I.partials + (size_t)(a.parity ^ 1) * I.pstride * kPartialStride;

    __shared__ RegState S;
    __shared__ Acc rows[31][16];
    __shared__ Acc tot[32];
    __shared__ int active;
    const DGeom sg = I.sg[l], kg = I.kg[l];
    const float4 *__restrict__ scan = I.scan[l];
    const float4 *__restrict__ kf = I.kf[l];
    const int npix = sg.rows * sg.cols;
    const int base = tile * (kBlock * K);

    // ---- issue the independent loads together: this launch's scan surfels,
    // the previous launch's block partials and the state
    float4 s2[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int p = base + k * kBlock + tid;
        s2[k] = p < npix ? scan[p] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    Acc px[29];
    load_partials<29, Acc>(part_in, a.prev_level >= 0 ? npartials_of(I.nblocks[a.prev_level]) : 0, px);
    if (tid == 0) S = *slot_in;
    __syncthreads();

    // ---- 0. the previous launch's update, solved identically by every block
    if (S.pending && !S.stop) {
        block_reduce<29, Acc>(px, rows, tot);
        if (tid == 0) gn_step<Acc>(a, tot, S);
    }
    if (tid == 0) {
        S.pending = 0;
        if (MODE == MODE_ITER && a.first_of_level) S.level_active = 1;
        if (MODE == MODE_EVAL && a.check_max_iters && !S.stop && S.level_active) S.status = UPS_MAX_ITERS;
        active = (MODE == MODE_EVAL) || (!S.stop && S.level_active);
    }
    __syncthreads();
    if (!active) {
        if (tile == 0 && tid == 0) *slot_out = S;
        return;
    }

    // ---- 1. association of K pixels per thread at the updated pose
    Rt32 T;
#pragma unroll
    for (int k = 0; k < 9; k++) T.r[k] = (float)S.R[k];
#pragma unroll
    for (int k = 0; k < 3; k++) T.t[k] = (float)S.t[k];
    float s[NV], c[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) s[v] = c[v] = 0.f;
#pragma unroll
    for (int k = 0; k < K; k++) {
        // the 64 pixels of a wavefront lie in one row (cols is a multiple of 64)
        const int pw = __builtin_amdgcn_readfirstlane(base + k * kBlock + (tid & ~63));
        if (pw >= npix) break;
        const int i = pw / sg.cols;
        const int j = base + k * kBlock + tid - i * sg.cols;
        const Pair pr = associate(sg, s2[k], i, j, kg, kf, T, a.d_max2, a.cos_theta);
        if (pr.inlier) {
            const float3 qn = cross3(pr.q, pr.n1);
            const float J[6] = {qn.x, qn.y, qn.z, pr.n1.x, pr.n1.y, pr.n1.z};
            int e = 0;
#pragma unroll
            for (int u = 0; u < 6; u++)
#pragma unroll
                for (int w = u; w < 6; w++) {
                    if (PREC == UPS_PREC_KAHAN_F64) kahan_add(s[e], c[e], J[u] * J[w]);
                    else s[e] += J[u] * J[w];
                    e++;
                }
#pragma unroll
            for (int u = 0; u < 6; u++) {
                if (PREC == UPS_PREC_KAHAN_F64) kahan_add(s[21 + u], c[21 + u], J[u] * pr.r);
                else s[21 + u] += J[u] * pr.r;
            }
            if (PREC == UPS_PREC_KAHAN_F64) kahan_add(s[27], c[27], pr.r * pr.r);
            else s[27] += pr.r * pr.r;
            s[28] += 1.f;
        }
        if (MODE == MODE_EVAL) {
            if (range_ok(sg, s2[k].w)) {
                s[29] += 1.f;
                const float t = pr.inlier ? fminf(pr.r * pr.r, a.tau2) : a.tau2;
                if (PREC == UPS_PREC_KAHAN_F64) kahan_add(s[30], c[30], t);
                else s[30] += t;
            }
        }
    }

    // ---- 2. block partial
    {
        Acc x[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) x[v] = (PREC == UPS_PREC_KAHAN_F64) ? (Acc)s[v] - (Acc)c[v] : (Acc)s[v];
        block_reduce<NV, Acc>(x, rows, tot);
    }
    if (tid < NV) part_out[(size_t)tile * kPartialStride + tid] = (double)tot[tid];
    if (tile == 0 && tid == 0) {
        S.pending = (MODE == MODE_ITER);
        S.npartials = ntiles;
        *slot_out = S;
    }
}

template <int K, int PREC, int MODE>
__global__ __launch_bounds__(kBlock) void k_icp_one(Inst I, StepArgs a) {
    icp_block<K, PREC, MODE>(I, a, blockIdx.x);
}

// Batch: block -> (registration, tile) by binary search in the level's prefix
// table of tile counts (tile_start[n] = total blocks).
template <int K, int PREC, int MODE>
__global__ __launch_bounds__(kBlock) void k_icp_batch(const Inst *__restrict__ insts,
                                                      const int *__restrict__ tile_start, int n, StepArgs a) {
    const int b = blockIdx.x;
    int lo = 0, hi = n;  // the last k with tile_start[k] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_start[mid] <= b) lo = mid;
        else hi = mid;
    }
    icp_block<K, PREC, MODE>(insts[lo], a, b - tile_start[lo]);
}

// One block: the evaluation partials -> result (quality at the final pose,
// plus the state's pose, status, iteration count and last step norm), or ->
// normal equations.
template <int PREC>
__device__ __forceinline__ void finish_block(const Inst &I, int parity) {
    using Acc = typename std::conditional<PREC == UPS_PREC_KAHAN_F64, double, float>::type;
    __shared__ Acc rows[31][16];
    __shared__ Acc tot[32];
    const RegState *S = I.state + parity;
    reduce_partials<31, Acc>(I.partials + (size_t)parity * I.pstride * kPartialStride, npartials_of(I.nblocks[0]),
                             rows, tot);
    if (threadIdx.x != 0) return;
    const double n_in = (double)tot[28], n_valid = (double)tot[29];
    if (I.res) {
        ups_icp_result *r = I.res;
        for (int k = 0; k < 9; k++) r->T.R[k] = S->R[k];
        for (int k = 0; k < 3; k++) r->T.t[k] = S->t[k];
        r->status = S->status;
        r->iters_run = S->iters_run;
        r->last_update_norm = S->last_norm;
        for (int k = 0; k < 21; k++) r->JtJ[k] = (double)tot[k];
        for (int k = 0; k < 6; k++) r->Jtr[k] = (double)tot[21 + k];
        r->inliers = (int64_t)n_in;
        r->valid = (int64_t)n_valid;
        r->inlier_ratio = n_valid > 0 ? n_in / n_valid : 0.0;
        r->rms = n_in > 0 ? sqrt((double)tot[27] / n_in) : 0.0;
        r->trunc_cost = (double)tot[30];
    }
    if (I.neq) {
        ups_normal_eq *q = I.neq;
        for (int k = 0; k < 21; k++) q->JtJ[k] = (double)tot[k];
        for (int k = 0; k < 6; k++) q->Jtr[k] = (double)tot[21 + k];
        q->sum_r2 = (double)tot[27];
        q->inliers = (int64_t)n_in;
        q->valid = (int64_t)n_valid;
    }
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_finish_one(Inst I, int parity) {
    finish_block<PREC>(I, parity);
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_finish_batch(const Inst *__restrict__ insts, int parity) {
    finish_block<PREC>(insts[blockIdx.x], parity);
}

// More than 256 partials: fold them into one before the next launch reads
// them (keeps the per-block read of step 0 bounded).
template <int PREC, int NV>
__global__ __launch_bounds__(kBlock) void k_collapse_one(Inst I, int parity) {
    using Acc = typename std::conditional<PREC == UPS_PREC_KAHAN_F64, double, float>::type;
    __shared__ Acc rows[NV][16];
    __shared__ Acc tot[32];
    RegState *S = I.state + parity;
    double *part = I.partials + (size_t)parity * I.pstride * kPartialStride;
    if (NV == 29 && !S->pending) return;
    reduce_partials<NV, Acc>(part, S->npartials, rows, tot);
    if (threadIdx.x < NV) part[threadIdx.x] = (double)tot[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) S->npartials = 1;
}

// ------------------------------------------------- pyramid + registration init

__global__ __launch_bounds__(kBlock) void k_prepare_one(Inst I, const ups_pose *init, int levels) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t == 0) {
        RegState S;
        memset(&S, 0, sizeof(S));
        for (int k = 0; k < 9; k++) S.R[k] = init->R[k];
        for (int k = 0; k < 3; k++) S.t[k] = init->t[k];
        S.status = UPS_CONVERGED;
        S.level_active = 1;
        I.state[0] = S;
    }
    // subsample levels 1.. of the scan (image 0) and the keyframe (image 1)
    int q = t;
    for (int img = 0; img < 2; img++) {
        const DGeom &g0 = img ? I.kg[0] : I.sg[0];
        const float4 *src = img ? I.kf[0] : I.scan[0];
        for (int l = 1; l < levels; l++) {
            const DGeom &gl = img ? I.kg[l] : I.sg[l];
            const int n = gl.rows * gl.cols;
            if (q < n) {
                const int i = q / gl.cols, j = q - i * gl.cols;
                float4 *dst = const_cast<float4 *>(img ? I.kf[l] : I.scan[l]);
                dst[q] = src[(size_t)(i << l) * g0.cols + (j << l)];
                return;
            }
            q -= n;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_subsample(const float4 *__restrict__ src, int cols0, int level,
                                                      int rows, int cols, float4 *__restrict__ dst) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= rows * cols) return;
    const int i = q / cols, j = q - i * cols;
    dst[q] = src[(size_t)(i << level) * cols0 + (j << level)];
}

ups_status launch_subsample(const DGeom &g0, const float4 *src, int level, float4 *dst, hipStream_t s) {
    const int rows = g0.rows >> level, cols = g0.cols >> level;
    const int n = rows * cols;
    hipLaunchKernelGGL(k_subsample, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, src, g0.cols, level, rows,
                       cols, dst);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

// -------------------------------------------------------------- launchers

// Pixels per thread for a single registration: as few as keep the block
// count at or below 256, so that step 0 reads at most 256 partials.
int pick_k_single(int npix) {
    int K = 1;
    while (K < 16 && (npix + kBlock * K - 1) / (kBlock * K) > 256) K *= 2;
    return K;
}

template <int PREC, int MODE>
static ups_status launch_one_k(int K, const Inst &I, const StepArgs &a, int blocks, hipStream_t s) {
    switch (K) {
#define UPS_K(k) \
    case k: hipLaunchKernelGGL((k_icp_one<k, PREC, MODE>), dim3(blocks), dim3(kBlock), 0, s, I, a); break;
        UPS_K(1) UPS_K(2) UPS_K(4) UPS_K(8) UPS_K(16)
#undef UPS_K
        default:
            set_error("unsupported pixels-per-thread");
            return UPS_ERR_INVALID_ARG;
    }
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

static ups_status launch_one(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                             hipStream_t s) {
    if (prec == UPS_PREC_KAHAN_F64)
        return mode == MODE_ITER ? launch_one_k<UPS_PREC_KAHAN_F64, MODE_ITER>(K, I, a, blocks, s)
                                 : launch_one_k<UPS_PREC_KAHAN_F64, MODE_EVAL>(K, I, a, blocks, s);
    return mode == MODE_ITER ? launch_one_k<UPS_PREC_F32, MODE_ITER>(K, I, a, blocks, s)
                             : launch_one_k<UPS_PREC_F32, MODE_EVAL>(K, I, a, blocks, s);
}

template <int K, int PREC, int MODE>
static void launch_batch_t(const Inst *insts, const int *tile_start, int n, const StepArgs &a, int blocks,
                           hipStream_t s) {
    hipLaunchKernelGGL((k_icp_batch<K, PREC, MODE>), dim3(blocks), dim3(kBlock), 0, s, insts, tile_start, n, a);
}

ups_status launch_icp_batch(int K, int prec, int mode, const Inst *insts, const int *tile_start, int n,
                            const StepArgs &a, int blocks, hipStream_t s) {
    bool ok = true;
    switch (K * 4 + prec * 2 + mode) {
#define UPS_B(k)                                                                                         \
    case k * 4 + UPS_PREC_KAHAN_F64 * 2 + MODE_ITER:                                                     \
        launch_batch_t<k, UPS_PREC_KAHAN_F64, MODE_ITER>(insts, tile_start, n, a, blocks, s);            \
        break;                                                                                           \
    case k * 4 + UPS_PREC_KAHAN_F64 * 2 + MODE_EVAL:                                                     \
        launch_batch_t<k, UPS_PREC_KAHAN_F64, MODE_EVAL>(insts, tile_start, n, a, blocks, s);            \
        break;                                                                                           \
    case k * 4 + UPS_PREC_F32 * 2 + MODE_ITER:                                                           \
        launch_batch_t<k, UPS_PREC_F32, MODE_ITER>(insts, tile_start, n, a, blocks, s);                  \
        break;                                                                                           \
    case k * 4 + UPS_PREC_F32 * 2 + MODE_EVAL:                                                           \
        launch_batch_t<k, UPS_PREC_F32, MODE_EVAL>(insts, tile_start, n, a, blocks, s);                  \
        break;
        UPS_B(1) UPS_B(2) UPS_B(4) UPS_B(8) UPS_B(16)
#undef UPS_B
        default:
            ok = false;
    }
    if (!ok) {
        set_error("unsupported pixels-per-thread / precision");
        return UPS_ERR_INVALID_ARG;
    }
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_finish_batch(int prec, const Inst *insts, int n, int parity, hipStream_t s) {
    if (prec == UPS_PREC_KAHAN_F64)
        hipLaunchKernelGGL(k_finish_batch<UPS_PREC_KAHAN_F64>, dim3(n), dim3(kBlock), 0, s, insts, parity);
    else
        hipLaunchKernelGGL(k_finish_batch<UPS_PREC_F32>, dim3(n), dim3(kBlock), 0, s, insts, parity);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

static ups_status launch_finish_one(int prec, const Inst &I, int parity, hipStream_t s) {
    if (prec == UPS_PREC_KAHAN_F64)
        hipLaunchKernelGGL(k_finish_one<UPS_PREC_KAHAN_F64>, dim3(1), dim3(kBlock), 0, s, I, parity);
    else
        hipLaunchKernelGGL(k_finish_one<UPS_PREC_F32>, dim3(1), dim3(kBlock), 0, s, I, parity);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

static ups_status launch_collapse_one(int prec, int mode, const Inst &I, int parity, hipStream_t s) {
    if (prec == UPS_PREC_KAHAN_F64) {
        if (mode == MODE_ITER)
            hipLaunchKernelGGL((k_collapse_one<UPS_PREC_KAHAN_F64, 29>), dim3(1), dim3(kBlock), 0, s, I, parity);
        else
            hipLaunchKernelGGL((k_collapse_one<UPS_PREC_KAHAN_F64, 31>), dim3(1), dim3(kBlock), 0, s, I, parity);
    } else {
        if (mode == MODE_ITER)
            hipLaunchKernelGGL((k_collapse_one<UPS_PREC_F32, 29>), dim3(1), dim3(kBlock), 0, s, I, parity);
        else
            hipLaunchKernelGGL((k_collapse_one<UPS_PREC_F32, 31>), dim3(1), dim3(kBlock), 0, s, I, parity);
    }
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

// A registration: prepare (init + pyramids), the Gauss-Newton launches level
// by level, the evaluation launch and the finish launch.  The descriptor
// carries the state/partials scratch; pixels per thread follow pick_k_single.
ups_status launch_register(const Inst &I0, const ups_pose *init, const ups_icp_params &p, hipStream_t s) {
    Inst I = I0;
    int Ks[4] = {1, 1, 1, 1};
    for (int l = 0; l < p.levels; l++) {
        const int npix = I.sg[l].rows * I.sg[l].cols;
        Ks[l] = pick_k_single(npix);
        I.nblocks[l] = (npix + kBlock * Ks[l] - 1) / (kBlock * Ks[l]);
    }
    int npre = 0;
    for (int l = 1; l < p.levels; l++) npre += I.sg[l].rows * I.sg[l].cols + I.kg[l].rows * I.kg[l].cols;
    const int pre_blocks = npre > 0 ? (npre + kBlock - 1) / kBlock : 1;
    hipLaunchKernelGGL(k_prepare_one, dim3(pre_blocks), dim3(kBlock), 0, s, I, init, p.levels);
    UPS_CHECK_HIP(hipGetLastError());

    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.cos_theta = p.cos_theta_max;
    a.min_inliers = p.min_inliers;
    a.stop_norm = p.stop_update_norm;
    int parity = 0;
    ups_status st;
    a.prev_level = -1;
    for (int l = p.levels - 1; l >= 0; l--) {
        a.level = l;
        a.d_max2 = p.d_max[l] * p.d_max[l];
        for (int it = 0; it < p.iters[l]; it++) {
            a.parity = parity;
            a.first_of_level = it == 0;
            if ((st = launch_one(Ks[l], p.precision, MODE_ITER, I, a, I.nblocks[l], s)) != UPS_OK) return st;
            a.prev_level = l;
            parity ^= 1;
            if (I.nblocks[l] > 256 && (st = launch_collapse_one(p.precision, MODE_ITER, I, parity, s)) != UPS_OK)
                return st;
        }
    }
    // evaluation at level 0: apply the last update, quality terms
    a.level = 0;
    a.parity = parity;
    a.first_of_level = 0;
    a.d_max2 = p.d_max[0] * p.d_max[0];
    a.tau2 = a.d_max2;
    a.check_max_iters = (p.stop_update_norm > 0.0 && p.iters[0] > 0);
    if ((st = launch_one(Ks[0], p.precision, MODE_EVAL, I, a, I.nblocks[0], s)) != UPS_OK) return st;
    parity ^= 1;
    if (I.nblocks[0] > 256 && (st = launch_collapse_one(p.precision, MODE_EVAL, I, parity, s)) != UPS_OK) return st;
    return launch_finish_one(p.precision, I, parity, s);
}

// Normal equations at a fixed pose: prepare (pose only) + evaluation + finish.
ups_status launch_eval(const Inst &I0, const ups_pose *T, float d_max, float cos_theta, int precision,
                       hipStream_t s) {
    Inst I = I0;
    const int npix = I.sg[0].rows * I.sg[0].cols;
    const int K = pick_k_single(npix);
    I.nblocks[0] = (npix + kBlock * K - 1) / (kBlock * K);
    hipLaunchKernelGGL(k_prepare_one, dim3(1), dim3(kBlock), 0, s, I, T, 1);
    UPS_CHECK_HIP(hipGetLastError());
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.level = 0;
    a.parity = 0;
    a.prev_level = -1;
    a.d_max2 = d_max * d_max;
    a.tau2 = a.d_max2;
    a.cos_theta = cos_theta;
    ups_status st = launch_one(K, precision, MODE_EVAL, I, a, I.nblocks[0], s);
    if (st != UPS_OK) return st;
    if (I.nblocks[0] > 256 && (st = launch_collapse_one(precision, MODE_EVAL, I, 1, s)) != UPS_OK) return st;
    return launch_finish_one(precision, I, 1, s);
}

// ---------------------------------------------------------- correspondences

__global__ __launch_bounds__(kBlock) void k_correspondences(DGeom sg, const float4 *__restrict__ scan, DGeom kg,
                                                            const float4 *__restrict__ kf, const ups_pose *pose,
                                                            float d_max2, float cos_theta, int32_t *idx,
                                                            uint8_t *inl) {
    const int npix = sg.rows * sg.cols;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const Rt32 T = load_pose_f32(pose);
    const int i = p / sg.cols, j = p - i * sg.cols;
    const Pair pr = associate(sg, scan[p], i, j, kg, kf, T, d_max2, cos_theta);
    idx[p] = pr.kf_index;
    inl[p] = pr.inlier ? 1 : 0;
}

ups_status launch_correspondences(const DGeom &sg, const float4 *scan, const DGeom &kg, const float4 *kf,
                                  const ups_pose *T, float d_max, float cos_theta, int32_t *idx, uint8_t *inl,
                                  hipStream_t s) {
    const int npix = sg.rows * sg.cols;
    hipLaunchKernelGGL(k_correspondences, dim3((npix + kBlock - 1) / kBlock), dim3(kBlock), 0, s, sg, scan, kg, kf,
                       T, d_max * d_max, cos_theta, idx, inl);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
