// Device code of the projective point-to-plane ICP (UPSLAM Section III-B,
// Equation 1): per-thread accumulation, block reductions, the FP64 solve and
// update, the iteration kernel and the batch solve / finish kernels.  The
// iteration kernel is instantiated per (pixels per thread, precision, mode,
// variant) in separate translation units (ups_icp_*.hip) so that they
// compile in parallel.
#pragma once

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

// Sums over lane groups by DPP: quad_sum over each quad (xor 1, xor 2),
// oct_sum over each group of 8 lanes (then the half-row mirror).  Every lane
// of a group ends with the bitwise-same sum (the two operands of each
// addition are the same pair in every lane, and addition commutes).
template <typename T>
__device__ __forceinline__ T quad_sum(T v) {
    if constexpr (sizeof(T) == 8) {
        v += dpp_d<0xB1>(v);
        v += dpp_d<0x4E>(v);
    } else {
        v += dpp_f<0xB1>(v);
        v += dpp_f<0x4E>(v);
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T oct_sum(T v) {
    v = quad_sum<T>(v);
    if constexpr (sizeof(T) == 8) v += dpp_d<0x141>(v);
    else v += dpp_f<0x141>(v);
    return v;
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float x) {
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Per-thread accumulation of the per-pixel terms in the three precision modes.
template <int PREC, int NV>
struct ThreadAcc;

// Compensated FP32 where it pays: the Gauss-Newton fixed point is where
// J^T r vanishes, so J^T r (values 21..26), sum r^2 (27) and the truncated
// cost (30) are Kahan-compensated; the 21 J^T J entries, whose rounding only
// perturbs the step size, are plain FP32 sums; counts are exact.  The
// compensated values are summed plainly over a group of up to 4 pixels and
// each group sum enters the Kahan sum (flush), which keeps the compensation
// at a quarter of the per-pixel cost; a 4-term FP32 sum adds at most 3 ulp
// of its terms' magnitude before compensation.
template <int NV>
struct ThreadAcc<UPS_PREC_KAHAN_F64, NV> {
    static constexpr int NC = NV > 30 ? 8 : 7;  // compensated values
    float s[NV], c[NC], g[NC];
    static __device__ __forceinline__ constexpr int comp(int v) { return (v >= 21 && v < 28) ? v - 21 : (v == 30 ? 7 : -1); }
    static __device__ __forceinline__ constexpr int value_of(int j) { return j < 7 ? 21 + j : 30; }
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int v = 0; v < NV; v++) s[v] = 0.f;
#pragma unroll
        for (int j = 0; j < NC; j++) c[j] = g[j] = 0.f;
    }
    __device__ __forceinline__ void add(int v, float x) {
        if (comp(v) >= 0) g[comp(v)] += x;
        else s[v] += x;
    }
    __device__ __forceinline__ void count(int v) { s[v] += 1.f; }
    // the group sums enter the compensated sums
    __device__ __forceinline__ void flush() {
#pragma unroll
        for (int j = 0; j < NC; j++) {
            kahan_add(s[value_of(j)], c[j], g[j]);
            g[j] = 0.f;
        }
    }
    __device__ __forceinline__ double get(int v) const {
        return comp(v) >= 0 ? (double)s[v] - (double)c[comp(v)] : (double)s[v];
    }
};

template <int NV>
struct ThreadAcc<UPS_PREC_F32, NV> {  // plain FP32
    float s[NV];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int v = 0; v < NV; v++) s[v] = 0.f;
    }
    __device__ __forceinline__ void add(int v, float x) { s[v] += x; }
    __device__ __forceinline__ void count(int v) { s[v] += 1.f; }
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ float get(int v) const { return s[v]; }
};

template <int NV>
struct ThreadAcc<UPS_PREC_F64, NV> {  // FP64 (callers add exact FP64 products)
    double s[NV];
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int v = 0; v < NV; v++) s[v] = 0.0;
    }
    __device__ __forceinline__ void add(int v, double x) { s[v] += x; }
    __device__ __forceinline__ void fma(int v, double a, double b) { s[v] = ::fma(a, b, s[v]); }
    __device__ __forceinline__ void count(int v) { s[v] += 1.0; }
    __device__ __forceinline__ void flush() {}
    __device__ __forceinline__ double get(int v) const { return s[v]; }
};

template <int PREC>
using AccOf = typename std::conditional<PREC == UPS_PREC_F32, float, double>::type;

// Add one inlier's 28 terms: the upper triangle of wt J^T J, wt J^T r and the
// unweighted r^2.  wt is the IRLS weight; the squared objective passes the
// constant 1, whose products fold away at compile time.
template <int PREC, int NV>
__device__ __forceinline__ void add_terms(ThreadAcc<PREC, NV> &acc, const Pair &pr, float wt) {
    const float3 qn = cross3(pr.q, pr.n1);
    if constexpr (PREC == UPS_PREC_F64) {
        const double J[6] = {qn.x, qn.y, qn.z, pr.n1.x, pr.n1.y, pr.n1.z};
        const double r = pr.r;
        double Jw[6];
#pragma unroll
        for (int u = 0; u < 6; u++) Jw[u] = J[u] * (double)wt;
        int e = 0;
#pragma unroll
        for (int u = 0; u < 6; u++)
#pragma unroll
            for (int w = u; w < 6; w++) acc.fma(e++, Jw[u], J[w]);
#pragma unroll
        for (int u = 0; u < 6; u++) acc.fma(21 + u, Jw[u], r);
        acc.fma(27, r, r);
    } else {
        const float J[6] = {qn.x, qn.y, qn.z, pr.n1.x, pr.n1.y, pr.n1.z};
        float Jw[6];
#pragma unroll
        for (int u = 0; u < 6; u++) Jw[u] = J[u] * wt;
        int e = 0;
#pragma unroll
        for (int u = 0; u < 6; u++)
#pragma unroll
            for (int w = u; w < 6; w++) acc.add(e++, Jw[u] * J[w]);
#pragma unroll
        for (int u = 0; u < 6; u++) acc.add(21 + u, Jw[u] * pr.r);
        acc.add(27, pr.r * pr.r);
    }
    acc.count(28);
}

// The block's sum of NV per-thread values, written as this block's partial
// (value v at part_out[v * pstride + tile]), in a fixed order: quad sums by
// DPP, the 64 quad sums of each value through LDS, then 8 threads per value
// (thread g adds quads g, g+8, ..., g+56 pairwise) and oct_sum.
// ------------------------------------- agent-coherent words (batch scheduler)
//
// Data that blocks of one launch hand to each other (block partials,
// registration state, jobs, counters) is read and written only through
// relaxed agent-scope atomics, which the hardware keeps coherent across the
// XCDs' L2 caches without writing back or invalidating them.  A writer orders
// its data before the word that publishes it by waiting for its stores to
// complete (wait_stores); a reader has the published word in hand before it
// loads the data.
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <typename T>
__device__ __forceinline__ T ld_coh(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_coh(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double ld_coh_d(const double *p) {
    return __longlong_as_double((long long)ld_coh((const unsigned long long *)p));
}

__device__ __forceinline__ void st_coh_d(double *p, double v) {
    st_coh((unsigned long long *)p, (unsigned long long)__double_as_longlong(v));
}

constexpr int kStateWords = (int)(sizeof(RegState) / 4);

// A registration state copied word by word by threads 0 .. kStateWords-1.
__device__ __forceinline__ void state_ld_coh(RegState &dst, const RegState *src) {
    if (threadIdx.x < kStateWords)
        ((uint32_t *)&dst)[threadIdx.x] = ld_coh(((const uint32_t *)src) + threadIdx.x);
}

__device__ __forceinline__ void state_st_coh(RegState *dst, const RegState &src) {
    if (threadIdx.x < kStateWords)
        st_coh(((uint32_t *)dst) + threadIdx.x, ((const uint32_t *)&src)[threadIdx.x]);
}

// WAVE0: the NV totals are staged in LDS (stage[NV]) and stored by the first
// wavefront as agent-coherent words.
template <int NV, typename Acc, bool WAVE0 = false>
__device__ __forceinline__ void block_partial(const Acc (&x)[NV], Acc (*qbuf)[65], double *part_out, int pstride,
                                              int tile, Acc *stage = nullptr) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const Acc y = quad_sum<Acc>(x[v]);
        if ((tid & 3) == 0) qbuf[v][tid >> 2] = y;
    }
    __syncthreads();
    const int v = min(tid >> 3, NV - 1), g = tid & 7;
    Acc y[8];
#pragma unroll
    for (int k = 0; k < 8; k++) y[k] = qbuf[v][g + 8 * k];
#pragma unroll
    for (int w = 4; w >= 1; w >>= 1)
#pragma unroll
        for (int k = 0; k < w; k++) y[k] += y[k + w];
    const Acc t = oct_sum<Acc>(y[0]);
    if constexpr (WAVE0) {
        if (g == 0 && (tid >> 3) < NV) stage[v] = t;
        __syncthreads();
        if (tid < NV) st_coh_d(part_out + (size_t)tid * pstride + tile, (double)stage[tid]);
    } else {
        if (g == 0 && (tid >> 3) < NV) part_out[(size_t)v * pstride + tile] = (double)t;
    }
}

// The block's sum of NV per-thread values through one LDS transpose (single
// registrations, one block per CU, so the 64 KB buffer costs no occupancy):
// every thread stores its NV values, then the 8 threads of value v add the
// 256 values in a fixed order -- thread g the 32 values of threads g, g + 8,
// ..., g + 248 as a pairwise tree -- and oct_sum combines the 8.  Rows are
// padded by 8 values so that a wavefront's reads spread over the banks.
// COH: the partial stored as agent-coherent words.
template <int NV, typename Acc, bool COH = false>
__device__ __forceinline__ void block_partial_lds(const Acc (&x)[NV], double *part_out, int pstride, int tile) {
    constexpr int kRow = kBlock + 8;
    __shared__ Acc buf[NV * kRow];
    const int tid = threadIdx.x;
#pragma unroll
    for (int v = 0; v < NV; v++) buf[v * kRow + tid] = x[v];
    __syncthreads();
    const int v = min(tid >> 3, NV - 1), g = tid & 7;
    Acc y[32];
#pragma unroll
    for (int k = 0; k < 32; k++) y[k] = buf[v * kRow + g + 8 * k];
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1)
#pragma unroll
        for (int k = 0; k < w; k++) y[k] += y[k + w];
    const Acc t = oct_sum<Acc>(y[0]);
    if (g == 0 && (tid >> 3) < NV) {
        if constexpr (COH) st_coh_d(part_out + (size_t)v * pstride + tile, (double)t);
        else part_out[(size_t)v * pstride + tile] = (double)t;
    }
}

typedef double v2d __attribute__((ext_vector_type(2)));

// Value v = tid / 8 (clamped to NV - 1) summed over the first n block
// partials by the 8 threads of a group: thread g loads blocks 2g + 16k and
// 2g + 16k + 1 (two blocks per 16-byte load, 16 loads in flight per 256
// partials) and adds the 32 values pairwise (the pair of load k, then the
// sixteen pair sums as a tree), chunk by chunk, then oct_sum.  Every thread
// of the group returns the same total, and every block that reads the same
// partials computes the same totals.
// NL: 16-byte loads in flight per thread (a chunk of 16 NL partials).
// COH: each pair as two agent-coherent 8-byte loads (partials that blocks of
// the same launch wrote), the same sums.
template <int NV, typename Acc, int NL = 16, bool COH = false>
__device__ __forceinline__ Acc sum_partials(const double *part, int pstride, int n) {
    const int v = min((int)(threadIdx.x >> 3), NV - 1), g = threadIdx.x & 7;
    const UPS_AS_GLOBAL double *pv = (const UPS_AS_GLOBAL double *)part + (size_t)v * pstride;
    const double *pc = part + (size_t)v * pstride;
    Acc t = 0;
    for (int b0 = 0; b0 < n; b0 += 16 * NL) {
        const int nk = min(NL, (n - b0 + 15) >> 4);  // block-uniform
        v2d x[NL];
#pragma unroll
        for (int k = 0; k < NL; k++) {
            // an index past the last partial is clamped into the row and its value unused
            x[k] = (v2d){0.0, 0.0};
            if (k < nk) {
                const int b = min(b0 + 16 * k + 2 * g, pstride - 2);
                if constexpr (COH) x[k] = (v2d){ld_coh_d(pc + b), ld_coh_d(pc + b + 1)};
                else x[k] = *(const UPS_AS_GLOBAL v2d *)(pv + b);
            }
        }
        Acc y[NL];
#pragma unroll
        for (int k = 0; k < NL; k++) {
            const int b = b0 + 16 * k + 2 * g;
            y[k] = ((b < n) ? (Acc)x[k].x : Acc(0)) + ((b + 1 < n) ? (Acc)x[k].y : Acc(0));
        }
#pragma unroll
        for (int w = NL / 2; w >= 1; w >>= 1)
#pragma unroll
            for (int k = 0; k < w; k++) y[k] += y[k + w];
        t += y[0];
    }
    return oct_sum<Acc>(t);
}

// The totals of the first n partials into tot[0 .. NV-1] (LDS), visible to
// the whole block on return.
template <int NV, typename Acc, int NL = 16>
__device__ __forceinline__ void reduce_partials(const double *part, int pstride, int n, Acc *tot) {
    const Acc t = sum_partials<NV, Acc, NL>(part, pstride, n);
    if ((threadIdx.x & 7) == 0 && (threadIdx.x >> 3) < NV) tot[threadIdx.x >> 3] = t;
    __syncthreads();
}

// --------------------------------------------------------- FP64 / FP32 solve

// 1 / sqrt(d) for d > 0 (normal range): in FP64 the hardware estimate
// refined by one Newton step y <- y + y (1 - d y^2) / 2, which about squares
// its relative error (e -> 1.5 e^2).  Measured on gfx950 over 2^20
// log-uniform d in [1e-12, 1e12]: estimate 5.2e-8 (2^-24.2) at most, after
// the step 4.1e-15 (2^-47.8) at most and 8e-17 median -- far below what the
// FP32 per-pixel terms leave in the normal equations.  In FP32 the plain
// quotient.
template <typename T>
__device__ __forceinline__ T inv_sqrt(T d) {
    if constexpr (sizeof(T) == 8) {
        const double y = __builtin_amdgcn_rsq(d);
        const double e = fma(-d * y, y, 1.0);
        return fma(0.5 * y, e, y);
    } else {
        return T(1) / sqrt(d);
    }
}

// Index of entry (i, j), i <= j, in the row-major upper triangle of a 6x6 matrix.
__device__ __forceinline__ int tri6(int i, int j) { return i * 6 - (i * (i - 1)) / 2 + (j - i); }

// xi = -A^-1 b for the symmetric A given by its row-major upper triangle A21:
// Cholesky column by column, then forward and back substitution.  A pivot
// <= 1e-12 x the largest diagonal entry (or no positive diagonal) makes the
// system DEGENERATE; the pivots are checked once after the factorisation (a
// failed pivot only yields values that are then discarded), so that no
// branch splits the dependent chain.
template <typename T>
__device__ int cholesky_solve6(const T *A21, const T *b, T *xi) {
    T L[6][6], inv[6];
    T maxd = 0;
    for (int a = 0; a < 6; a++) {
        const T v = A21[tri6(a, a)];
        maxd = v > maxd ? v : maxd;
    }
    bool ok = maxd > T(0);
    for (int c = 0; c < 6; c++) {
        T d = A21[tri6(c, c)];
        for (int k = 0; k < c; k++) d -= L[c][k] * L[c][k];
        ok = ok && (d > T(1e-12) * maxd);
        inv[c] = inv_sqrt<T>(d);  // 1 / L[c][c]
        for (int r = c + 1; r < 6; r++) {
            T s = A21[tri6(c, r)];
            for (int k = 0; k < c; k++) s -= L[r][k] * L[c][k];
            L[r][c] = s * inv[c];
        }
    }
    if (!ok) return UPS_DEGENERATE;
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
// th^10 term (the first omitted term, th^12/13! for the first coefficient, is
// below 1e-17, a tenth of an ulp of its value near 1), which avoids the
// cancellation of the closed forms and any sin/cos; above it the closed forms
// are used.
template <typename T>
__device__ void exp_compose(const T *xi, double *R, double *t) {
    const T w0 = xi[0], w1 = xi[1], w2 = xi[2];
    const T th2 = w0 * w0 + w1 * w1 + w2 * w2;
    T A, B, C;
    if (th2 < T(0.0625)) {
        // 1/n! for n = 0..13
        constexpr double f[14] = {1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040,
                                  1.0 / 40320, 1.0 / 362880, 1.0 / 3628800, 1.0 / 39916800, 1.0 / 479001600,
                                  1.0 / 6227020800.0};
        A = B = C = 0;
        for (int k = 5; k >= 0; k--) {
            const T sg = (k & 1) ? T(-1) : T(1);
            A = A * th2 + sg * (T)f[2 * k + 1];
            B = B * th2 + sg * (T)f[2 * k + 2];
            C = C * th2 + sg * (T)f[2 * k + 3];
        }
    } else {
        const T th = sqrt(th2);
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
    S.level_iters[a.prev_level] += 1;
    T nrm = 0;
    for (int k = 0; k < 6; k++) nrm += xi[k] * xi[k];
    S.last_norm = (double)sqrt(nrm);
    if (a.stop_norm > 0.0 && S.last_norm < a.stop_norm) S.level_active = 0;
}

// -------------------------------------------- wavefront-parallel FP64 solve

// v as held by lane `lane` (the same lane in every lane of the wavefront).
template <typename T>
__device__ __forceinline__ T lane_bcast(T v, int lane) {
    if constexpr (sizeof(T) == 8) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
        return __hiloint2double(hi, lo);
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
    }
}

// v as held by lane src (a lane of its own for every lane, 0 <= src < 64).
template <typename T>
__device__ __forceinline__ T lane_fetch(T v, int src) {
    if constexpr (sizeof(T) == 8) {
        const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
        const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
        return __hiloint2double(hi, lo);
    } else {
        return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
    }
}

// Gauss-Newton step from the reduced totals (J^T J upper triangle in tot[0..20],
// J^T r in tot[21..26], inlier count in tot[28]), computed by one whole
// wavefront: every lane of it calls this with the same arguments.  The same
// update as gn_step with a few registers per lane instead of the whole 6x6
// factor in one thread's (the persistent batch kernel, whose occupancy the
// solve's registers would otherwise set); slower on its own than gn_step,
// whose chain of FP64 operations has no cross-lane waits.  Lane 6r+c
// holds entry (r, c) of the 6x6 matrix.  Cholesky column by column (pivot
// broadcast from its lane, column scaled by the pivot's inverse square root,
// trailing entries updated with the column's values fetched from their lanes:
// the same operations in the same order as the textbook column loop), then
// forward and back substitution for xi = -A^-1 b with the right-hand side in
// lanes 0..5, then T <- Exp(xi) T with one output entry per lane (R in lanes
// 0..8, t in lanes 9..11).  A pivot <= 1e-12 x the largest diagonal entry,
// or fewer than min_inliers inliers, stops the registration with the pose
// unchanged.  Lane 0 updates the iteration counts, the step norm and the
// level's convergence.  S is the block's state copy (LDS).
template <typename T>
__device__ void gn_step_wave(const StepArgs &a, const T *tot, RegState &S) {
    const int lane = threadIdx.x & 63;
    if ((double)tot[28] < (double)a.min_inliers) {
        if (lane == 0) {
            S.status = UPS_NO_INLIERS;
            S.stop = 1;
        }
        return;
    }
    const int r = lane / 6, c = lane - 6 * (lane / 6);
    const bool mat = lane < 36;
    T x = mat ? tot[r <= c ? tri6(r, c) : tri6(c, r)] : T(0);
    T maxd = 0;
#pragma unroll
    for (int d = 0; d < 6; d++) {
        const T v = tot[tri6(d, d)];
        maxd = v > maxd ? v : maxd;
    }
    bool ok = maxd > T(0);
    T inv[6];
#pragma unroll
    for (int j = 0; j < 6; j++) {
        const T d = lane_bcast(x, 7 * j);
        ok = ok && d > T(1e-12) * maxd;
        inv[j] = ok ? inv_sqrt<T>(d) : T(0);
        if (c == j && r >= j) x *= inv[j];  // column j of L (the pivot becomes sqrt(d))
        const T lr = lane_fetch(x, min(6 * r + j, 63)), lc = lane_fetch(x, min(6 * c + j, 63));
        if (mat && r > j && c > j) x -= lr * lc;
    }
    if (!ok) {
        if (lane == 0) {
            S.status = UPS_DEGENERATE;
            S.stop = 1;
        }
        return;
    }
    // forward substitution L y = -b (lane i < 6 holds row i), then L^T xi = y
    T z = lane < 6 ? -tot[21 + lane] : T(0);
    {
        T Lrow[6];
#pragma unroll
        for (int j = 0; j < 6; j++) Lrow[j] = lane_fetch(x, min(6 * lane + j, 63));  // L[lane][j]
#pragma unroll
        for (int j = 0; j < 6; j++) {
            if (lane == j) z *= inv[j];
            const T yj = lane_bcast(z, j);
            if (lane > j && lane < 6) z -= Lrow[j] * yj;
        }
    }
    T Lcol[6];
#pragma unroll
    for (int j = 0; j < 6; j++) Lcol[j] = lane_fetch(x, min(6 * j + lane, 63));  // L[j][lane]
    T xi[6];
#pragma unroll
    for (int j = 5; j >= 0; j--) {
        if (lane == j) z *= inv[j];
        xi[j] = lane_bcast(z, j);
        if (lane < j) z -= Lcol[j] * xi[j];
    }
    // T <- Exp(xi) T: Rodrigues rotation E and the V matrix; below |omega| =
    // 1/4 the coefficients sin(th)/th, (1-cos th)/th^2 and (th-sin th)/th^3
    // from their Taylor series to the th^10 term (the first omitted term,
    // th^12/13! for the first, is below 1e-17), else the closed forms
    const T w0 = xi[0], w1 = xi[1], w2 = xi[2];
    const T th2 = w0 * w0 + w1 * w1 + w2 * w2;
    T A, B, C;
    if (th2 < T(0.0625)) {
        // 1/n! for n = 0..13
        constexpr double f[14] = {1.0, 1.0, 1.0 / 2, 1.0 / 6, 1.0 / 24, 1.0 / 120, 1.0 / 720, 1.0 / 5040,
                                  1.0 / 40320, 1.0 / 362880, 1.0 / 3628800, 1.0 / 39916800, 1.0 / 479001600,
                                  1.0 / 6227020800.0};
        A = B = C = 0;
#pragma unroll
        for (int k = 5; k >= 0; k--) {
            const T sg = (k & 1) ? T(-1) : T(1);
            A = A * th2 + sg * (T)f[2 * k + 1];
            B = B * th2 + sg * (T)f[2 * k + 2];
            C = C * th2 + sg * (T)f[2 * k + 3];
        }
    } else {
        const T th = sqrt(th2);
        A = sin(th) / th;
        B = (T(1) - cos(th)) / th2;
        C = (th - sin(th)) / (th2 * th);
    }
    const T K[3][3] = {{0, -w2, w1}, {w2, 0, -w0}, {-w1, w0, 0}};
    const int row = lane < 9 ? lane / 3 : (lane < 12 ? lane - 9 : 0);
    T E[3], V[3];
#pragma unroll
    for (int m = 0; m < 3; m++) {
        T K2 = 0;
#pragma unroll
        for (int q = 0; q < 3; q++) K2 += (row == 0 ? K[0][q] : row == 1 ? K[1][q] : K[2][q]) * K[q][m];
        const T Krm = row == 0 ? K[0][m] : row == 1 ? K[1][m] : K[2][m];
        const T I = (row == m) ? T(1) : T(0);
        E[m] = I + A * Krm + B * K2;
        V[m] = I + B * Krm + C * K2;
    }
    T out = 0;
    if (lane < 9) {
        const int col = lane - 3 * row;
        out = E[0] * (T)S.R[col] + E[1] * (T)S.R[3 + col] + E[2] * (T)S.R[6 + col];
    } else if (lane < 12) {
        const T te = V[0] * xi[3] + V[1] * xi[4] + V[2] * xi[5];
        out = E[0] * (T)S.t[0] + E[1] * (T)S.t[1] + E[2] * (T)S.t[2] + te;
    }
    // every lane has read the old pose before any lane writes the new one
    __builtin_amdgcn_wave_barrier();
    if (lane < 9) S.R[lane] = (double)out;
    else if (lane < 12) S.t[lane - 9] = (double)out;
    if (lane == 0) {
        S.iters_run += 1;
        S.level_iters[a.prev_level] += 1;
        T nrm = 0;
#pragma unroll
        for (int k = 0; k < 6; k++) nrm += xi[k] * xi[k];
        S.last_norm = (double)sqrt(nrm);
        if (a.stop_norm > 0.0 && S.last_norm < a.stop_norm) S.level_active = 0;
    }
}

// ------------------------------------------------------------------ kernel

// Partials a launch over `nblocks` blocks leaves for its successor: one per
// block, or a single folded one when there are more than 256.
__device__ __host__ __forceinline__ int npartials_of(int nblocks) { return nblocks > 256 ? 1 : nblocks; }

// FUSED: the block first applies the previous launch's update itself (step 0
// above; single registrations and the batch's main loop), with the state and
// partials in ping-pong slots (a.parity).  Otherwise (the batch's subset and
// scheduled paths) another launch has already applied it and left the pose,
// and whether this launch has work for the registration, in state slot 0.
// STRIDED: level l is read from the level-0 images, every 2^l-th row and
// column (single registrations); otherwise from the level's pyramid images.
// WORLD: the world-frame variant (state pose = the scan's world pose).
// IRLS: the absolute-value objective of Equation 1, each inlier's terms
// weighted by 1 / max(|r|, a.irls_delta).
// COH (FUSED only): the state and the partials are read and written as
// agent-coherent words, for blocks of one launch that hand them to each other
// (the one-XCD level kernel); the same values as the plain accesses.
// The state a registration starts from: the start pose (world-frame variant:
// the scan's world pose, keyframe world pose x start pose, in FP64), status
// CONVERGED, the first level active, no iterations run.
__device__ __forceinline__ void init_state(const Inst &I, const ups_pose *init, RegState &S) {
    memset(&S, 0, sizeof(S));
    if (I.world) {
        for (int a = 0; a < 3; a++) {
            for (int c = 0; c < 3; c++)
                S.R[3 * a + c] =
                    I.wR[3 * a] * init->R[c] + I.wR[3 * a + 1] * init->R[3 + c] + I.wR[3 * a + 2] * init->R[6 + c];
            S.t[a] = I.wR[3 * a] * init->t[0] + I.wR[3 * a + 1] * init->t[1] + I.wR[3 * a + 2] * init->t[2] + I.wt[a];
        }
    } else {
        for (int k = 0; k < 9; k++) S.R[k] = init->R[k];
        for (int k = 0; k < 3; k++) S.t[k] = init->t[k];
    }
    S.status = UPS_CONVERGED;
    S.level_active = 1;
}

// Phase timestamps of single-registration launches, in the instrumented build
// only (UPS_PHASE_TIMESTAMPS, compiled into the translation unit that defines
// UPS_PHASE_TU and the arrays): for launch a.seq of a call, the 100 MHz
// real-time clock when tile 0's thread 0 enters, has the previous partials
// reduced, has solved, has finished its pixels and has stored its partial,
// plus the earliest entry and the latest exit over all blocks.
#if defined(UPS_PHASE_TIMESTAMPS) && defined(UPS_PHASE_TU)
constexpr int kPhaseLaunches = 64;
extern __device__ unsigned long long g_phase_mark[kPhaseLaunches][5];
extern __device__ unsigned long long g_phase_first[kPhaseLaunches];
extern __device__ unsigned long long g_phase_last[kPhaseLaunches];
#define UPS_PHASE(FUSED_, TILE_, SEQ_, K_)                                                                 \
    do {                                                                                                 \
        if ((FUSED_) && (TILE_) == 0 && threadIdx.x == 0 && (SEQ_) >= 0 && (SEQ_) < kPhaseLaunches)      \
            g_phase_mark[SEQ_][K_] = __builtin_amdgcn_s_memrealtime();                                   \
    } while (0)
#define UPS_PHASE_FIRST(FUSED_, SEQ_)                                                                    \
    do {                                                                                                 \
        if ((FUSED_) && threadIdx.x == 0 && (SEQ_) >= 0 && (SEQ_) < kPhaseLaunches)                      \
            atomicMin(&g_phase_first[SEQ_], __builtin_amdgcn_s_memrealtime());                          \
    } while (0)
#define UPS_PHASE_LAST(FUSED_, SEQ_)                                                                     \
    do {                                                                                                 \
        if ((FUSED_) && threadIdx.x == 0 && (SEQ_) >= 0 && (SEQ_) < kPhaseLaunches)                      \
            atomicMax(&g_phase_last[SEQ_], __builtin_amdgcn_s_memrealtime());                            \
    } while (0)
#else
#define UPS_PHASE(FUSED_, TILE_, SEQ_, K_) do {} while (0)
#define UPS_PHASE_FIRST(FUSED_, SEQ_) do {} while (0)
#define UPS_PHASE_LAST(FUSED_, SEQ_) do {} while (0)
#endif

// LDS workspace of one block's tile (one per kernel, whichever modes it runs).
template <typename Acc>
struct IcpShared {
    RegState S;
    Acc qbuf[31][65];
    Acc tot[32];
    int active;
    int job[8];  // persistent scheduler: ticket's registration and tile, last-arriver flag, spare, job (4 words)
};

template <int K, int PREC, int MODE, bool FUSED, bool WORLD, bool IRLS, bool STRIDED = FUSED, bool COH = false>
__device__ __forceinline__ void icp_tile(const Inst &I, const StepArgs &a, int tile, IcpShared<AccOf<PREC>> &sh) {
    static_assert(!COH || (FUSED && MODE == MODE_ITER), "coherent hand-over: fused iterations only");
    constexpr int NV = (MODE == MODE_EVAL) ? 31 : 29;  // EVAL adds valid count and truncated cost
    using Acc = AccOf<PREC>;
    const int tid = threadIdx.x;
    const int l = a.level;
    const int ntiles = I.nblocks[l];
    RegState *slot_in = I.state + (FUSED ? a.parity : 0), *slot_out = I.state + (a.parity ^ 1);
    const double *part_in = I.partials + (size_t)a.parity * I.pstride * kPartialStride;
    double *part_out = I.partials + (size_t)(FUSED ? (a.parity ^ 1) : 0) * I.pstride * kPartialStride;

    [[maybe_unused]] constexpr bool kPh = FUSED && STRIDED;  // phase timestamps: single registrations
    UPS_PHASE_FIRST(kPh, a.seq);
    UPS_PHASE(kPh, tile, a.seq, 0);
    RegState &S = sh.S;
    Acc(&qbuf)[31][65] = sh.qbuf;
    Acc(&tot)[32] = sh.tot;
    int &active = sh.active;
    const DGeom sg = I.sg[l], kg = I.kg[l];
    const int ish = STRIDED ? l : 0;
    const float4 *__restrict__ scan = I.scan[STRIDED ? 0 : l];
    const float4 *__restrict__ kf = I.kf[STRIDED ? 0 : l];
    const int npix = sg.rows * sg.cols;
    // scan image index of level-l pixel q, whose wavefront starts at pixel qw
    // (wave-uniform) and whose column is jcol; past the last pixel: clamped
    // into the image
    auto scan_index = [&](int q, int qw, int jcol) -> uint32_t {
        if constexpr (STRIDED) {
            const int row = __builtin_amdgcn_readfirstlane(min(qw, npix - 1)) / sg.cols;
            return (uint32_t)((row * (sg.cols << ish) + jcol) << ish);
        } else {
            return (uint32_t)min(q, npix - 1);
        }
    };
    // pixels per thread of this tile: K, or fewer for a scheduled tile
    const int KL = (MODE == MODE_SCHED) ? a.kpt : K;
    const int base = tile * (kBlock * KL);

    // ---- issue the independent loads together: the first pair of scan
    // surfels and their ray-table columns, the previous launch's block
    // partials and the state.  Scan loads are clamped into the image (the last
    // wavefronts of a tile may run past it) and masked afterwards, so no load
    // sits behind a branch.  Pixels go in pairs: both pixels' keyframe gathers
    // are in flight before the first of them is consumed, and the next pair's
    // scan loads behind them.
    constexpr int P = (K >= 2) ? 2 : 1;
    const int pw0 = __builtin_amdgcn_readfirstlane(base + (tid & ~63));
    // column of this thread's pixel; it advances by kBlock mod cols per pixel
    const int col_step = kBlock % sg.cols;
    float4 nx[P];
    float2 na[P];
    int jc[P];
#pragma unroll
    for (int u = 0; u < P; u++) {
        if (u == 0) jc[u] = (base + tid) % sg.cols;
        else jc[u] = jc[u - 1] + col_step >= sg.cols ? jc[u - 1] + col_step - sg.cols : jc[u - 1] + col_step;
        nx[u] = ldg_u(scan, scan_index(base + u * kBlock + tid, pw0 + u * kBlock, jc[u]));
        na[u] = ldg_u(sg.lut_col, (uint32_t)jc[u] << sg.lshift);
    }
    if (!FUSED) {
        if (MODE == MODE_ITER && !slot_in->active) return;  // uniform: the whole block leaves
        if (MODE == MODE_EVAL && slot_in->skip) return;
        if constexpr (MODE == MODE_SCHED) state_ld_coh(S, slot_in);
        else if (tid == 0) S = *slot_in;
        __syncthreads();
    } else {
        // the state, one 32-bit word per thread, loaded alongside the partials
        static_assert(sizeof(RegState) % 4 == 0 && kStateWords <= kBlock, "state copy");
        uint32_t sword = 0;
        if (tid < kStateWords)
            sword = COH ? ld_coh((const uint32_t *)slot_in + tid) : ((const UPS_AS_GLOBAL uint32_t *)slot_in)[tid];
        const Acc ptot = sum_partials<29, Acc, 16, COH>(part_in, I.pstride,
                                                        a.prev_level >= 0 ? npartials_of(I.nblocks[a.prev_level]) : 0);
        if (tid < kStateWords) ((uint32_t *)&S)[tid] = sword;
        if ((tid & 7) == 0 && (tid >> 3) < 29) tot[tid >> 3] = ptot;
        __syncthreads();
        UPS_PHASE(kPh, tile, a.seq, 1);
        // ---- 0. the previous launch's update, solved identically by every block
        // (the first launch of a call: the state from the start pose)
        if (tid == 0) {
            if (a.init) init_state(I, a.init, S);
            if (S.pending && !S.stop) gn_step<Acc>(a, tot, S);
            S.pending = 0;
            if (MODE == MODE_ITER && a.first_of_level) S.level_active = 1;
            if (MODE == MODE_EVAL && a.check_max_iters && !S.stop && S.level_active) S.status = UPS_MAX_ITERS;
            active = (MODE == MODE_EVAL) || (!S.stop && S.level_active);
        }
        __syncthreads();
        UPS_PHASE(kPh, tile, a.seq, 2);
        if (!active) {
            if (tile == 0 && tid == 0) *slot_out = S;
            return;
        }
    }

    // ---- 1. association of K pixels per thread at the updated pose (the pose
    // is block-uniform: kept in scalar registers)
    Rt32 T;
#pragma unroll
    for (int k = 0; k < 9; k++) T.r[k] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int((float)S.R[k])));
#pragma unroll
    for (int k = 0; k < 3; k++) T.t[k] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int((float)S.t[k])));
    Rt32 Wk;
    if constexpr (WORLD) {
#pragma unroll
        for (int k = 0; k < 9; k++) Wk.r[k] = (float)I.wR[k];
#pragma unroll
        for (int k = 0; k < 3; k++) Wk.t[k] = (float)I.wt[k];
    }
    ThreadAcc<PREC, NV> acc;
    acc.zero();
    int pw = pw0;
    // groups of up to 4 pixels (the Kahan group).  From 8 pixels per thread
    // on, one group per trip of a loop that is not unrolled (unrolled, the
    // 32-pixel batch kernel is 118 KB of code, more than the instruction cache
    // holds); below, two groups per trip, so that the compensated sums need
    // no register copies between trips
    constexpr int GP = K < 4 ? K : 4;
    constexpr int kGroupUnroll = K >= 8 ? 1 : 2;
    bool done = false;
#pragma unroll kGroupUnroll
    for (int k0 = 0; k0 < KL; k0 += GP) {
#pragma unroll
        for (int k = k0; k < k0 + GP; k += P) {
            if (pw >= npix) {
                done = true;
                break;
            }
            Gather G[P];
            float sw[P];
#pragma unroll
            for (int u = 0; u < P; u++) {
                const float4 s2 = make_float4(nx[u].x, nx[u].y, nx[u].z,
                                              (base + (k + u) * kBlock + tid < npix) ? nx[u].w : 0.f);
                sw[u] = s2.w;
                const int i = min(pw + u * kBlock, npix - 1) / sg.cols;
                const float2 e = lds_uniform(sg.lut_row, i * sg.stride);
                if constexpr (WORLD) G[u] = scan_side_world(sg, s2, e, na[u], kg, kf, T, Wk, ish);
                else G[u] = scan_side(sg, s2, e, na[u], kg, kf, T, ish);
                // keep the consumers of these gathers below the next pixel's scan side
                __builtin_amdgcn_sched_barrier(0);
            }
            {
                const bool more = k + P < KL;
#pragma unroll
                for (int u = 0; u < P; u++) {
                    jc[u] += more ? P * col_step : 0;
                    jc[u] = jc[u] >= sg.cols ? jc[u] - sg.cols : jc[u];
                    jc[u] = jc[u] >= sg.cols ? jc[u] - sg.cols : jc[u];
                    const int ku = more ? k + P + u : k + u;
                    nx[u] = ldg_u(scan, scan_index(base + ku * kBlock + tid, pw + (ku - k) * kBlock, jc[u]));
                    na[u] = ldg_u(sg.lut_col, (uint32_t)jc[u] << sg.lshift);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < P; u++) {
                bool inl;
                float r;
                float3 n1;
                if constexpr (WORLD) kf_side_world(kg, G[u], Wk, a.d_max2, a.cos_theta, inl, r, n1);
                else kf_side(kg, G[u], a.d_max2, a.cos_theta, inl, r, n1);
                if (inl) {
                    Pair pr;
                    pr.inlier = true;
                    pr.r = r;
                    pr.q = G[u].q;
                    pr.n1 = n1;
                    float wt = 1.f;
                    if constexpr (IRLS) wt = __builtin_amdgcn_rcpf(fmaxf(fabsf(r), a.irls_delta));
                    add_terms<PREC, NV>(acc, pr, wt);
                }
                if (MODE == MODE_EVAL) {
                    if (range_ok(sg, sw[u])) {
                        acc.count(29);
                        acc.add(30, inl ? fminf(r * r, a.tau2) : a.tau2);
                    }
                }
            }
            pw = __builtin_amdgcn_readfirstlane(pw + P * kBlock);
        }
        acc.flush();
        if (done) break;
    }

    UPS_PHASE(kPh, tile, a.seq, 3);
    // ---- 2. block partial
    {
        Acc x[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) x[v] = (Acc)acc.get(v);
        if constexpr (STRIDED && MODE != MODE_SCHED)
            block_partial_lds<NV, Acc, COH>(x, part_out, I.pstride, tile);
        else
            block_partial<NV, Acc, MODE == MODE_SCHED>(x, qbuf, part_out, I.pstride, tile, tot);
    }
    UPS_PHASE(kPh, tile, a.seq, 4);
    if (FUSED && tile == 0) {
        if (tid == 0) {
            S.pending = (MODE == MODE_ITER);
            S.npartials = ntiles;
            if (!COH) *slot_out = S;
        }
        if constexpr (COH) {
            __syncthreads();
            state_st_coh(slot_out, S);
        }
    }
    UPS_PHASE_LAST(kPh, a.seq);
}

template <int K, int PREC, int MODE, bool FUSED, bool WORLD, bool IRLS, bool STRIDED = FUSED>
__device__ __forceinline__ void icp_block(const Inst &I, const StepArgs &a, int tile) {
    __shared__ IcpShared<AccOf<PREC>> sh;
    icp_tile<K, PREC, MODE, FUSED, WORLD, IRLS, STRIDED>(I, a, tile, sh);
}

// Workgroups are dealt to the 8 XCDs in turn (workgroup i to XCD i mod 8), and
// each XCD has its own L2: the tiles are permuted so that the workgroups of
// one XCD take a contiguous run of tiles, and neighbouring tiles of a
// registration, whose keyframe gathers share cache lines, meet in one L2.
// Any other dealing still covers every tile once; the debug order reverses
// it (the partials are reduced in tile order, so results do not change).
__device__ __forceinline__ int xcd_tile(int blk, int nblk, int reverse) {
    const int x = blk & 7, q = blk >> 3, per = nblk >> 3, rem = nblk & 7;
    const int t = x < rem ? x * (per + 1) + q : rem * (per + 1) + (x - rem) * per + q;
    return reverse ? nblk - 1 - t : t;
}

template <int K, int PREC, int MODE, bool WORLD, bool IRLS>
__global__ __launch_bounds__(kBlock) void k_icp_one(Inst I, StepArgs a) {
    // the one-XCD level kernels' counters (a pair per level), zero again for
    // the next call (those kernels, if they ran, ended before this launch)
    if (blockIdx.x == 0 && threadIdx.x < 8 && I.xsync) I.xsync[threadIdx.x] = 0;
    icp_block<K, PREC, MODE, true, WORLD, IRLS>(I, a, xcd_tile(blockIdx.x, gridDim.x, a.reverse_tiles));
}

// All `iters` Gauss-Newton iterations of one pyramid level of a single
// registration in one launch, its tiles on one XCD.  Workgroups are dealt to
// the 8 XCDs in turn; a workgroup reads its XCD from the hardware and those
// on XCD `xcd_sel` take tickets (the tiles, in order) until the level's tiles
// are taken; all others leave.  The host rotates xcd_sel from launch to
// launch, so that level kernels running at once on several streams wait on
// different XCDs (each XCD holds the workgroups of two of them at a time).  Between iterations the tiles hand their block
// partials and the state to each other as agent-coherent words (a CU's L1
// keeps lines across a workgroup-scope invalidate, so plain loads could
// return what the same CU read an iteration earlier): every wavefront waits
// for its stores, the workgroup counts itself in an atomic counter, polls it
// (atomic adds of `zero`, never served from L1) until all tiles have arrived
// and goes on with the next iteration, whose prologue reads the partials and
// applies the update exactly as a separate launch would (the same sums,
// bitwise the same result).  A level that converges or a registration
// that stops ends the loop in every workgroup at once (they hold the same
// state).  The last iteration's partials are left for the next launch; the
// state goes to the slot that launch reads, (a.parity + iters) mod 2.  A
// workgroup whose unsuccessful polls exceed spin_limit in all (the level's
// workgroups could not all run on the chosen XCD at once) gives up rather than waiting
// on: it sets the counter's top bit, so every other workgroup gives up at its
// next poll and the launch ends, and it overwrites its partial of the level's
// last iteration with NaN, which the launch that reads it turns into the
// DEGENERATE status (its solve finds no positive pivot).  Tile 0 giving up
// stores the DEGENERATE state itself; either way the registration never goes
// on from a sum that lacks a tile.  Each level has its own pair of counters; the
// per-iteration and evaluation launches after this one zero them.
constexpr unsigned kLevelGaveUp = 1u << 31;  // arrival counter bit: a workgroup gave up

template <int K, int PREC, bool WORLD, bool IRLS>
__global__ __launch_bounds__(kBlock) void k_icp_level_xcd(Inst I, StepArgs a, int iters, unsigned xcd_sel,
                                                          unsigned zero, unsigned spin_limit) {
    __shared__ IcpShared<AccOf<PREC>> sh;
    __shared__ int ticket_s, fail_s;
    const int tid = threadIdx.x;
    const int ntiles = I.nblocks[a.level];
    unsigned *const tickets = I.xsync + 2 * a.level, *const arrivals = tickets + 1;  // this level's pair
    if (tid == 0) {
        const unsigned xcd = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 0xFu;  // HW_REG_XCC_ID, bits 3:0
        int t = -1;
        if (xcd == xcd_sel) {
            const unsigned k = __hip_atomic_fetch_add(tickets, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (k < (unsigned)ntiles) t = (int)k;
        }
        ticket_s = t;
        fail_s = 0;
    }
    __syncthreads();
    const int ticket = ticket_s;
    if (ticket < 0) return;
    const int tile = a.reverse_tiles ? ntiles - 1 - ticket : ticket;
    unsigned spins = 0;
    for (int it = 0; it < iters; it++) {
        StepArgs ai = a;
        ai.parity = (a.parity + it) & 1;
        ai.seq = a.seq + it;
        if (it > 0) {
            ai.first_of_level = 0;
            ai.prev_level = a.level;
            ai.init = nullptr;
        }
        icp_tile<K, PREC, MODE_ITER, true, WORLD, IRLS, true, true>(I, ai, tile, sh);
        if (!sh.active) break;  // converged or stopped: the same decision in every workgroup
        if (it + 1 == iters) break;  // the last iteration's partials are the next launch's
        // this workgroup's partial (and tile 0's state) stores completed, then its arrival
        wait_stores();
        __syncthreads();
        if (tid == 0) {
            __hip_atomic_fetch_add(arrivals, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = (unsigned)ntiles * (unsigned)(it + 1);
            for (;;) {
                const unsigned v = __hip_atomic_fetch_add(arrivals, zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (v & kLevelGaveUp) {  // another workgroup gave up: so does this one
                    fail_s = 1;
                    break;
                }
                if (v >= target) break;
                if (++spins > spin_limit) {
                    fail_s = 1;
                    __hip_atomic_fetch_or(arrivals, kLevelGaveUp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        if (fail_s) break;
    }
    if (fail_s) {
        double *last = I.partials + (size_t)((a.parity + iters) & 1) * I.pstride * kPartialStride;
        if (tid < kPartialStride)
            st_coh_d(last + (size_t)tid * I.pstride + tile, __longlong_as_double(0x7ff8000000000000ll));
        if (tid == 0) {
            sh.S.stop = 1;
            sh.S.pending = 0;
            sh.S.status = UPS_DEGENERATE;
        }
    }
    __syncthreads();
    if (tile == 0 && tid == 0) I.state[(a.parity + iters) & 1] = sh.S;
}

// Batch: block -> (registration, tile) from the level's table a.tile_of (one
// load), or by binary search in the level's prefix table of tile counts
// (tile_start[n] = total blocks; a chain of dependent loads at the head of
// every block).  FUSED: each block first applies its registration's pending
// update (the batch's main loop); otherwise slot 0 holds the pose (the
// subset and scheduled paths, timing).
template <int K, int PREC, int MODE, bool IRLS, bool FUSED>
__global__ __launch_bounds__(kBlock) void k_icp_batch(const Inst *__restrict__ insts,
                                                      const int *__restrict__ tile_start, int n, StepArgs a) {
    const int b = xcd_tile(blockIdx.x, gridDim.x, a.reverse_tiles);
    if (a.tile_of) {
        const unsigned v = a.tile_of[b];
        icp_block<K, PREC, MODE, FUSED, false, IRLS, false>(insts[v >> 16], a, (int)(v & 0xFFFFu));
        return;
    }
    int lo = 0, hi = n;  // the last k with tile_start[k] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_start[mid] <= b) lo = mid;
        else hi = mid;
    }
    icp_block<K, PREC, MODE, FUSED, false, IRLS, false>(insts[lo], a, b - tile_start[lo]);
}

// A subset of the batch (a Compact list), in the main loop's fused form: a
// fixed grid strides over the subset's tiles, so the launch costs little when
// the subset is small, and each tile first applies its registration's
// pending update (state and partials in ping-pong slots, a.parity).
template <int K, int PREC, int MODE, bool IRLS>
__global__ __launch_bounds__(kBlock) void k_icp_batch_list(const Inst *__restrict__ insts,
                                                           const Compact *__restrict__ hdr,
                                                           const int *__restrict__ list,
                                                           const int *__restrict__ start, StepArgs a) {
    const int cnt = hdr->count, total = hdr->total[a.level];
    for (int t0 = blockIdx.x; t0 < total; t0 += gridDim.x) {
        const int t = a.reverse_tiles ? total - 1 - t0 : t0;
        int lo = 0, hi = cnt;  // the last m with start[m] <= t
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (start[mid] <= t) lo = mid;
            else hi = mid;
        }
        __syncthreads();  // the previous tile's state copy (LDS) is no longer read
        icp_block<K, PREC, MODE, true, false, IRLS, false>(insts[list[lo]], a, t - start[lo]);
    }
}


// One block: the evaluation partials -> result (quality at the final pose,
// plus the state's pose, status, iteration count and last step norm), or ->
// normal equations.
template <typename Acc>
__device__ void write_result(const Inst &I, const RegState *S, const Acc *tot, ups_icp_result *res,
                             ups_normal_eq *neq);

template <int PREC>
__device__ __forceinline__ void finish_block(const Inst &I, int parity, ups_icp_result *res, ups_normal_eq *neq) {
    using Acc = AccOf<PREC>;
    __shared__ Acc tot[32];
    const RegState *S = I.state + parity;
    if (S->skip) return;  // masked out of this batch call: the result is left as it was
    reduce_partials<31, Acc>(I.partials + (size_t)parity * I.pstride * kPartialStride, I.pstride,
                             npartials_of(I.nblocks[0]), tot);
    write_result<Acc>(I, S, tot, res, neq);
}

// The result of a registration (quality at the final pose from the 31
// evaluation totals, plus the state's pose, status, iteration counts and last
// step norm), or its normal equations; called by every thread of the block,
// each writing a few of the fields.
template <typename Acc>
__device__ void write_result(const Inst &I, const RegState *S, const Acc *tot, ups_icp_result *res,
                             ups_normal_eq *neq) {
    const int t = threadIdx.x;
    if (t < 27) {
        const double v = (double)tot[t];
        if (res) (t < 21 ? res->JtJ[t] : res->Jtr[t - 21]) = v;
        if (neq) (t < 21 ? neq->JtJ[t] : neq->Jtr[t - 21]) = v;
    }
    if (res && t >= 32 && t < 44) {
        const int k = t - 32;  // entry of the pose: R row-major (0..8), then t (9..11)
        double v;
        if (I.world) {
            // scan -> keyframe = (keyframe world pose)^-1 (scan world pose), FP64
            if (k < 9) {
                const int a = k / 3, c = k - 3 * (k / 3);
                v = I.wR[a] * S->R[c] + I.wR[3 + a] * S->R[3 + c] + I.wR[6 + a] * S->R[6 + c];
            } else {
                const int a = k - 9;
                v = I.wR[a] * (S->t[0] - I.wt[0]) + I.wR[3 + a] * (S->t[1] - I.wt[1]) +
                    I.wR[6 + a] * (S->t[2] - I.wt[2]);
            }
        } else {
            v = k < 9 ? S->R[k] : S->t[k - 9];
        }
        if (k < 9) res->T.R[k] = v;
        else res->T.t[k - 9] = v;
    }
    if (t == 64) {
        const double n_in = (double)tot[28], n_valid = (double)tot[29];
        if (res) {
            res->status = S->status;
            res->iters_run = S->iters_run;
            for (int k = 0; k < 4; k++) res->level_iters[k] = S->level_iters[k];
            res->last_update_norm = S->last_norm;
            res->inliers = (int64_t)n_in;
            res->valid = (int64_t)n_valid;
            res->inlier_ratio = n_valid > 0 ? n_in / n_valid : 0.0;
            res->rms = n_in > 0 ? sqrt((double)tot[27] / n_in) : 0.0;
            res->trunc_cost = (double)tot[30];
        }
        if (neq) {
            neq->sum_r2 = (double)tot[27];
            neq->inliers = (int64_t)n_in;
            neq->valid = (int64_t)n_valid;
        }
    }
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_finish_one(Inst I, int parity) {
    finish_block<PREC>(I, parity, I.res, I.neq);
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_finish_batch(const Inst *__restrict__ insts, int parity,
                                                         ups_icp_result *results) {
    finish_block<PREC>(insts[blockIdx.x], parity, results + blockIdx.x, nullptr);
}

// The results of the registrations of a Compact list only, a small grid
// striding over them.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_finish_batch_list(const Inst *__restrict__ insts,
                                                              const Compact *__restrict__ hdr,
                                                              const int *__restrict__ list, int parity,
                                                              ups_icp_result *results) {
    const int cnt = hdr->count;
    for (int m = blockIdx.x; m < cnt; m += gridDim.x) {
        __syncthreads();  // the previous registration's totals (LDS) are no longer read
        finish_block<PREC>(insts[list[m]], parity, results + list[m], nullptr);
    }
}

// More than 256 iteration partials: fold them into one before the next
// launch reads them (keeps the per-block read of step 0 bounded).
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_collapse_one(Inst I, int parity) {
    constexpr int NV = 29;
    using Acc = AccOf<PREC>;
    RegState *S = I.state + parity;
    double *part = I.partials + (size_t)parity * I.pstride * kPartialStride;
    if (!S->pending) return;
    // the 8 threads of value v read only row v, and have read all of it
    // before the group's sum exists: the total can overwrite block 0's entry
    const Acc t = sum_partials<NV, Acc>(part, I.pstride, S->npartials);
    if ((threadIdx.x & 7) == 0 && (threadIdx.x >> 3) < NV) part[(size_t)(threadIdx.x >> 3) * I.pstride] = (double)t;
    __syncthreads();
    if (threadIdx.x == 0) S->npartials = 1;
}


// Value v = tid / 8 (clamped to NV - 1) summed over the first n block
// partials through agent-coherent loads: thread g of the group adds partials
// g, g + 8, ... in order, then oct_sum; the totals into tot (LDS), visible
// to the whole block on return.  The same sums whatever the blocks' order of
// arrival.  All 32 loads of a chunk of 256 partials are issued before the
// first is added (one memory round trip per chunk).
template <int NV, typename Acc>
__device__ __forceinline__ void reduce_partials_coh(const double *part, int pstride, int n, Acc *tot) {
    const int v = min((int)(threadIdx.x >> 3), NV - 1), g = threadIdx.x & 7;
    const double *pv = part + (size_t)v * pstride;
    Acc t = 0;
    for (int b0 = 0; b0 < n; b0 += 256) {
        // an index past the last partial is clamped and its value unused
        double x[32];
#pragma unroll
        for (int q = 0; q < 32; q++) x[q] = ld_coh_d(pv + min(b0 + g + 8 * q, n - 1));
#pragma unroll
        for (int q = 0; q < 32; q++) t += (b0 + g + 8 * q < n) ? (Acc)x[q] : Acc(0);
    }
    t = oct_sum<Acc>(t);
    if ((threadIdx.x & 7) == 0 && (threadIdx.x >> 3) < NV) tot[threadIdx.x >> 3] = t;
    __syncthreads();
}

// ------------------------------------------------- persistent batch scheduler
//
// One launch runs every registration of a batch call through its
// Gauss-Newton iterations.  Each registration has one job in flight (an
// iteration at a level); a job's tiles carry consecutive ticket numbers,
// recorded in the tile map with the call's epoch and the job's level.  A
// worker block takes the next ticket, waits until its tile is published,
// processes it (the iteration kernel's tile body), writes its block partial
// and counts itself in the registration's arrivals.  The block that completes
// a job reduces the job's partials in tile order (the same sums whatever the
// order of arrival), applies the update in FP64 and publishes the next job,
// or, after the last iteration, counts the registration out.  Registrations
// that converge stop publishing, so the launch's work follows the active
// registrations.  A worker leaves when every registration is done, or, as a
// last resort against a broken protocol, after kSpinLimit polls (error flag).
// Everything blocks hand to each other goes through agent-coherent words
// (ld_coh / st_coh), published after wait_stores.  The evaluation at the final
// poses is the launch that follows.

// polls of a waiting worker before it gives up (each after a short sleep;
// seconds in all, while normal waits are microseconds)
constexpr unsigned kSpinLimit = 1u << 22;

__device__ __forceinline__ int sched_ntiles(const SchedArgs &A, const Inst &I, int level) {
    const int np = I.sg[level].rows * I.sg[level].cols, K = A.kpt[level];
    return (np + kBlock * K - 1) / (kBlock * K);
}

// The first job: the coarsest level with iterations, else the evaluation.
__device__ __forceinline__ SchedJob first_job(const SchedArgs &A, const Inst &I) {
    int l = A.levels - 1;
    while (l >= 0 && A.iters[l] == 0) l--;
    SchedJob J;
    J.level = l >= 0 ? l : 0;
    J.mode = l >= 0 ? MODE_ITER : MODE_EVAL;
    J.iter = 0;
    J.ntiles = sched_ntiles(A, I, J.level);
    return J;
}

// The job after J, given the state S after J's update: the next iteration of
// the level while it has not converged, else the first iteration of the next
// finer level with iterations, else the evaluation.  As in the launch
// sequence: a level that converged or a registration that stopped skips its
// remaining iterations; MAX_ITERS when a stop criterion is set and level 0
// ends without meeting it.
__device__ __forceinline__ SchedJob next_job(const SchedArgs &A, const Inst &I, const SchedJob &J, RegState &S) {
    SchedJob N;
    N.iter = 0;
    if (!S.stop && S.level_active && J.iter + 1 < A.iters[J.level]) {
        N.level = J.level;
        N.mode = MODE_ITER;
        N.iter = J.iter + 1;
    } else {
        int l = J.level - 1;
        while (l >= 0 && A.iters[l] == 0) l--;
        if (!S.stop && l >= 0) {
            S.level_active = 1;
            N.level = l;
            N.mode = MODE_ITER;
        } else {
            if (J.level == 0 && A.stop_norm > 0.0 && !S.stop && S.level_active) S.status = UPS_MAX_ITERS;
            N.level = 0;
            N.mode = MODE_EVAL;
        }
    }
    N.ntiles = sched_ntiles(A, I, N.level);
    S.active = N.mode == MODE_ITER;
    return N;
}

// Tile-map word of a job's tiles (the tile index goes in bits 0..9):
// epoch << 32 | mode << 31 | level << 29 | registration << 10.
__device__ __forceinline__ unsigned long long sched_tag(unsigned epoch, int k, const SchedJob &J) {
    return ((unsigned long long)epoch << 32) | ((unsigned long long)(unsigned)J.mode << 31) |
           ((unsigned long long)(unsigned)J.level << 29) | ((unsigned long long)(unsigned)k << 10);
}

// The block that finished job J of registration k: reduce the job's partials,
// then either update the registration and publish its next job, or write its
// result and count it out.  Not inlined: it runs once per job, and inlined
// into the tile loop its registers would lower the worker's occupancy.
template <int PREC>
__device__ __noinline__ void sched_complete(const SchedArgs &A, const Inst &I, int k, const SchedJob &J,
                                            unsigned epoch, IcpShared<AccOf<PREC>> &sh) {
    using Acc = AccOf<PREC>;
    RegState &S = sh.S;  // the tile's copy is free again
    reduce_partials_coh<29, Acc>(I.partials, I.pstride, J.ntiles, sh.tot);
    state_ld_coh(S, I.state);
    if (threadIdx.x == 0) sh.job[6] = ld_coh(&A.jobs[k].iter);  // the iteration within the level
    __syncthreads();
    {
        if (threadIdx.x < 64 && !S.stop) {
            StepArgs a;
            memset(&a, 0, sizeof(a));
            a.prev_level = J.level;
            a.min_inliers = A.min_inliers;
            a.stop_norm = A.stop_norm;
            gn_step_wave<Acc>(a, sh.tot, S);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            SchedJob Jc = J;
            Jc.iter = sh.job[6];
            const SchedJob N = next_job(A, I, Jc, S);
            sh.job[4] = N.level;
            sh.job[5] = N.mode;
            sh.job[6] = N.iter;
            sh.job[7] = N.ntiles;
        }
        __syncthreads();
        // the new state, job and arrival count, then their tiles; after the
        // last iteration the registration is done (the evaluation launch
        // that follows this kernel takes its final state)
        state_st_coh(I.state, S);
        const bool done = sh.job[5] == MODE_EVAL;
        unsigned base = 0;
        if (threadIdx.x == 0) {
            int *jw = (int *)(A.jobs + k);
            for (int q = 0; q < 4; q++) st_coh(jw + q, sh.job[4 + q]);
            st_coh(A.arrived + k, 0);
            // the new job's tickets, reserved while the stores complete
            if (!done)
                base = __hip_atomic_fetch_add(&A.sched->published, (unsigned)sh.job[7], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        }
        if (threadIdx.x < 64) wait_stores();  // the first wavefront wrote all of them
        if (threadIdx.x == 0 && done) {
            __hip_atomic_fetch_add(&A.sched->outstanding, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (threadIdx.x == 0) {
            const int nt = sh.job[7];
            if (base + (unsigned)nt > (unsigned)A.map_size) st_coh(&A.sched->error, 1);
            SchedJob N;
            N.level = sh.job[4];
            N.mode = sh.job[5];
            const unsigned long long tag = sched_tag(epoch, k, N);
            for (int i = 0; i < nt; i++)
                if (base + i < (unsigned)A.map_size) st_coh(A.tile_map + base + i, tag | (unsigned)i);
        }
    }
}

// The persistent worker (grid = the blocks that fit on the device at once).
// Thread 0 holds the ticket the block works on next: it takes it when it
// starts a tile and polls it after the tile (the first poll issued beside the
// tile's arrival), so the ticket's round trips overlap the tile's work.
template <int K, int PREC, bool IRLS>
__global__ __launch_bounds__(kBlock) void k_icp_persistent(SchedArgs A, const Inst *__restrict__ insts) {
    using Acc = AccOf<PREC>;
    __shared__ IcpShared<Acc> sh;
    const unsigned epoch = A.sched->epoch;
    unsigned t_next = 0;          // thread 0: the next ticket
    unsigned long long v_first = 0;  // thread 0: its first poll, issued with the arrival
    if (threadIdx.x == 0) t_next = __hip_atomic_fetch_add(&A.sched->next_ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (threadIdx.x == 0) {
            int k = -1, tile = 0, level = 0, mode = 0;
            const unsigned t = t_next;
            if (t < (unsigned)A.map_size) {
                // relaxed polls: no cache maintenance while waiting
                for (unsigned spin = 0;; spin++) {
                    const unsigned long long v = spin == 0 && v_first != 0 ? v_first : ld_coh(A.tile_map + t);
                    if ((unsigned)(v >> 32) == epoch) {
                        k = (int)((v >> 10) & 0xFFFFu);
                        tile = (int)(v & 1023u);
                        level = (int)((v >> 29) & 3u);
                        mode = (int)((v >> 31) & 1u);
                        break;
                    }
                    if ((spin & 15u) == 15u && ld_coh(&A.sched->outstanding) <= 0) {
                        // every registration is done: no tile will be published under this ticket
                        break;
                    }
                    if (spin >= kSpinLimit) {
                        st_coh(&A.sched->error, 1);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            if (k >= 0)
                t_next = __hip_atomic_fetch_add(&A.sched->next_ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh.job[0] = k;
            sh.job[1] = tile;
            sh.job[4] = level;
            sh.job[5] = mode;
        }
        __syncthreads();
        // wave-uniform: the registration's descriptor then comes through scalar loads
        const int k = __builtin_amdgcn_readfirstlane(sh.job[0]), tile = __builtin_amdgcn_readfirstlane(sh.job[1]);
        if (k < 0) return;  // block-uniform
        const Inst &I = insts[k];
        SchedJob J;
        J.level = __builtin_amdgcn_readfirstlane(sh.job[4]);
        J.mode = __builtin_amdgcn_readfirstlane(sh.job[5]);
        J.iter = 0;  // read from the job record by the block that completes the job
        J.ntiles = sched_ntiles(A, I, J.level);
        StepArgs a;
        memset(&a, 0, sizeof(a));
        a.level = J.level;
        a.prev_level = -1;
        a.d_max2 = A.d_max2[J.level];
        a.tau2 = A.d_max2[0];
        a.cos_theta = A.cos_theta;
        a.irls_delta = A.irls_delta;
        a.min_inliers = A.min_inliers;
        a.stop_norm = A.stop_norm;
        a.kpt = A.kpt[J.level];
        icp_tile<K, PREC, MODE_SCHED, false, false, IRLS>(I, a, tile, sh);
        // the tile's partial (stored by the first wavefront) before its arrival
        if (threadIdx.x < 64) {
            wait_stores();
            if (threadIdx.x == 0) {
                const int old = __hip_atomic_fetch_add(A.arrived + k, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                v_first = t_next < (unsigned)A.map_size ? ld_coh(A.tile_map + t_next) : 0ull;
                sh.job[2] = old == J.ntiles - 1;
            }
        }
        __syncthreads();
        if (sh.job[2]) {
            sched_complete<PREC>(A, I, k, J, epoch, sh);
            if (threadIdx.x == 0) v_first = 0;  // the block published tiles: poll afresh
        }
        __syncthreads();
    }
}

// Compile-time dispatch of (pixels per thread, precision, mode).
#define UPS_CASE_K(KV, ...)         \
    case KV: {                      \
        constexpr int KK = KV;      \
        __VA_ARGS__;                \
    } break;
#define UPS_DISPATCH_K(K, ...)                                                                            \
    switch (K) {                                                                                          \
        UPS_CASE_K(1, __VA_ARGS__) UPS_CASE_K(2, __VA_ARGS__) UPS_CASE_K(4, __VA_ARGS__)                  \
        UPS_CASE_K(8, __VA_ARGS__) UPS_CASE_K(16, __VA_ARGS__) UPS_CASE_K(32, __VA_ARGS__)                \
        UPS_CASE_K(64, __VA_ARGS__)                                                                       \
        default:                                                                                          \
            set_error("unsupported pixels-per-thread");                                                   \
            return UPS_ERR_INVALID_ARG;                                                                   \
    }
#define UPS_CASE_P(PV, ...)         \
    case PV: {                      \
        constexpr int PP = PV;      \
        __VA_ARGS__;                \
    } break;
#define UPS_DISPATCH_P(P, ...)                                                                            \
    switch (P) {                                                                                          \
        UPS_CASE_P(UPS_PREC_KAHAN_F64, __VA_ARGS__)                                                       \
        UPS_CASE_P(UPS_PREC_F32, __VA_ARGS__) UPS_CASE_P(UPS_PREC_F64, __VA_ARGS__)                       \
        default:                                                                                          \
            set_error("unknown precision mode");                                                          \
            return UPS_ERR_INVALID_ARG;                                                                   \
    }

}  // namespace ups
