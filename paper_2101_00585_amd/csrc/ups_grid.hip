// Loop-closure grid search (UPSLAM Section III-C): a few hundred candidate
// transforms of every registration of a batch are compared by a coarse
// projective alignment test -- the number of Omega inliers at a subsampled
// pyramid level -- and the best candidate becomes the start of the
// full-resolution registration.
//
// Candidates: c = (a, u, v) with yaw index a < n_yaw and grid indices
// u, v < n_xy; G_c = (Rz(2 pi a / n_yaw), ((u - h) s, (v - h) s, 0)) with
// h = (n_xy - 1) / 2 and s the grid step; the scored pose is base_k G_c.
//
// Scores are integer sums (block counts added with atomics), so they do not
// depend on the order in which blocks finish.
#include "ups_icp.hpp"

namespace ups {

// Candidate pose base * G_c in FP64 (row-major R, then t).
__device__ __forceinline__ void candidate_pose(const ups_pose &base, const GridArgs &g, int c, double *R,
                                               double *t) {
    const int per_yaw = g.n_xy * g.n_xy;
    const int a = c / per_yaw, u = (c / g.n_xy) % g.n_xy, v = c % g.n_xy;
    const double yaw = 6.283185307179586 * (double)a / (double)g.n_yaw;
    const double h = 0.5 * (double)(g.n_xy - 1);
    const double cy = cos(yaw), sy = sin(yaw);
    const double Gr[9] = {cy, -sy, 0.0, sy, cy, 0.0, 0.0, 0.0, 1.0};
    const double Gt[3] = {((double)u - h) * g.xy_step, ((double)v - h) * g.xy_step, 0.0};
    for (int r = 0; r < 3; r++) {
        for (int q = 0; q < 3; q++)
            R[3 * r + q] = base.R[3 * r] * Gr[q] + base.R[3 * r + 1] * Gr[3 + q] + base.R[3 * r + 2] * Gr[6 + q];
        t[r] = base.R[3 * r] * Gt[0] + base.R[3 * r + 1] * Gt[1] + base.R[3 * r + 2] * Gt[2] + base.t[r];
    }
}

// blockIdx.x: a tile of the batch at the grid level (the level's prefix table
// of tiles of kBlock * K pixels); blockIdx.y: the candidate.
__global__ __launch_bounds__(kBlock) void k_grid_score(const Inst *__restrict__ insts,
                                                       const int *__restrict__ tile_start, int n, int K,
                                                       const ups_pose *__restrict__ base, GridArgs g,
                                                       int *__restrict__ scores) {
    __shared__ float Ts[12];
    __shared__ int block_count;
    const int b = blockIdx.x, c = blockIdx.y, tid = threadIdx.x;
    int lo = 0, hi = n;  // the last k with tile_start[k] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_start[mid] <= b) lo = mid;
        else hi = mid;
    }
    const Inst &I = insts[lo];
    const int tile = b - tile_start[lo];
    const int l = g.level;
    const DGeom sg = I.sg[l], kg = I.kg[l];
    const float4 *__restrict__ scan = I.scan[l];
    const float4 *__restrict__ kf = I.kf[l];
    if (tid == 0) {
        double R[9], t[3];
        candidate_pose(base[lo], g, c, R, t);
        for (int q = 0; q < 9; q++) Ts[q] = (float)R[q];
        for (int q = 0; q < 3; q++) Ts[9 + q] = (float)t[q];
        block_count = 0;
    }
    __syncthreads();
    Rt32 T;
#pragma unroll
    for (int q = 0; q < 9; q++) T.r[q] = Ts[q];
#pragma unroll
    for (int q = 0; q < 3; q++) T.t[q] = Ts[9 + q];
    const int npix = sg.rows * sg.cols;
    int count = 0;
    for (int k = 0; k < K; k++) {
        // the 64 pixels of a wavefront lie in one row (cols is a multiple of 64)
        const int pw = __builtin_amdgcn_readfirstlane(tile * kBlock * K + k * kBlock + (tid & ~63));
        if (pw >= npix) break;
        const int p = pw + (tid & 63);
        const int i = pw / sg.cols, j = p - i * sg.cols;
        float4 s2 = ldg_u(scan, (uint32_t)min(p, npix - 1));
        s2.w = p < npix ? s2.w : 0.f;
        const float2 e = lds_uniform(sg.lut_row, i << sg.lshift);
        const float2 ca = ldg_u(sg.lut_col, (uint32_t)j << sg.lshift);
        const Gather G = scan_side(sg, s2, e, ca, kg, kf, T);
        bool inl;
        float r;
        float3 n1;
        kf_side(kg, G, g.d_max2, g.cos_theta, inl, r, n1);
        count += inl ? 1 : 0;
    }
    if (count) atomicAdd(&block_count, count);
    __syncthreads();
    if (tid == 0 && block_count) atomicAdd(&scores[lo * g.C + c], block_count);
}

// The scoring kernel for n_xy <= 5: blockIdx.x = a chunk of YB yaws (all
// NXY^2 translations of each), blockIdx.y = a tile of the level.  The scan
// pixels of the tile are loaded once per block and the rotated point and
// normal once per yaw; each candidate then costs a translation, the
// projection, the keyframe gathers and the Omega test.  Inlier counts are wave
// ballots accumulated in wave-uniform registers.  The same FP32 pose values
// and operations as k_grid_score, so the scores are the same.  Consecutive
// blocks share a tile, so its keyframe image is fetched into L2 once for all
// chunks that run together.
template <int NXY, int YB>
__global__ __launch_bounds__(kBlock) void k_grid_score_yaw(const Inst *__restrict__ insts,
                                                           const int *__restrict__ tile_start, int n, int K,
                                                           const ups_pose *__restrict__ base, GridArgs g,
                                                           int *__restrict__ scores) {
    constexpr int NT = NXY * NXY;
    __shared__ float Rs[YB][9];
    __shared__ float Ts[NT][3];
    __shared__ int wcount[kBlock / 64][YB * NT];
    const int chunk = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int lo = 0, hi = n;  // the last k with tile_start[k] <= b
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_start[mid] <= b) lo = mid;
        else hi = mid;
    }
    const Inst &I = insts[lo];
    const int tile = b - tile_start[lo];
    const int l = g.level;
    const DGeom sg = I.sg[l], kg = I.kg[l];
    const float4 *__restrict__ scan = I.scan[l];
    const float4 *__restrict__ kf = I.kf[l];
    const int a0 = chunk * YB;
    const int ny = min(YB, g.n_yaw - a0);  // yaws of this chunk
    // the FP64 candidate poses of candidate_pose, split: rotation base.R Rz(yaw)
    // per yaw, translation base.R Gt + base.t per grid cell, each rounded to FP32
    if (tid < ny) {
        double R[9], t[3];
        candidate_pose(base[lo], g, (a0 + tid) * NT, R, t);
        for (int q = 0; q < 9; q++) Rs[tid][q] = (float)R[q];
    }
    if (tid >= 64 && tid < 64 + NT) {
        double R[9], t[3];
        candidate_pose(base[lo], g, tid - 64, R, t);
        for (int q = 0; q < 3; q++) Ts[tid - 64][q] = (float)t[q];
    }
    __syncthreads();
    int cnt[YB * NT];
#pragma unroll
    for (int c = 0; c < YB * NT; c++) cnt[c] = 0;
    const int npix = sg.rows * sg.cols;
    for (int k = 0; k < K; k++) {
        // the 64 pixels of a wavefront lie in one row (cols is a multiple of 64)
        const int pw = __builtin_amdgcn_readfirstlane(tile * kBlock * K + k * kBlock + (tid & ~63));
        if (pw >= npix) break;
        const int p = pw + lane;
        const int i = pw / sg.cols, j = p - i * sg.cols;
        float4 s2 = ldg_u(scan, (uint32_t)min(p, npix - 1));
        s2.w = p < npix ? s2.w : 0.f;
        const float2 e = lds_uniform(sg.lut_row, i << sg.lshift);
        const float2 ca = ldg_u(sg.lut_col, (uint32_t)j << sg.lshift);
        const bool sok = surfel_ok(sg, s2);
        const float3 u = make_float3(e.x * ca.x, e.x * ca.y, e.y);
        const float3 p3 = make_float3(s2.w * u.x, s2.w * u.y, s2.w * u.z);
        const float3 n2 = make_float3(s2.x, s2.y, s2.z);
#pragma unroll
        for (int y = 0; y < YB; y++) {
            if (y >= ny) break;
            Rt32 T;
#pragma unroll
            for (int q = 0; q < 9; q++) T.r[q] = Rs[y][q];
            const float3 rp = rotate(T, p3);
            Gather G;
            G.m = rotate(T, n2);
#pragma unroll
            for (int t = 0; t < NT; t++) {
                G.q = make_float3(rp.x + Ts[t][0], rp.y + Ts[t][1], rp.z + Ts[t][2]);
                int ki, kj;
                const bool ok = project(kg, G.q, ki, kj) & sok;
                ki = ok ? ki : 0;
                kj = ok ? kj : 0;
                const uint32_t idx = __umul24((uint32_t)ki, (uint32_t)kg.cols) + (uint32_t)kj;
                G.kf_index = ok ? (int)idx : -1;
                G.s1 = ldg_u(kf, idx);
                G.e = ldg_u(kg.lut_row, (uint32_t)ki << kg.lshift);
                G.a = ldg_u(kg.lut_col, (uint32_t)kj << kg.lshift);
                bool inl;
                float r;
                float3 n1;
                kf_side(kg, G, g.d_max2, g.cos_theta, inl, r, n1);
                cnt[y * NT + t] += __builtin_popcountll(__builtin_amdgcn_ballot_w64(inl));
            }
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < YB * NT; c++) wcount[wave][c] = cnt[c];
    }
    __syncthreads();
    if (tid < ny * NT) {
        int s = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; w++) s += wcount[w][tid];
        if (s) atomicAdd(&scores[lo * g.C + a0 * NT + tid], s);
    }
}

__global__ void k_grid_zero(int *__restrict__ scores, int total) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) scores[i] = 0;
}

// One block per registration: the candidate with the most inliers (the
// lowest index among equals) and its pose.
__global__ __launch_bounds__(256) void k_grid_best(int C, const int *__restrict__ scores,
                                                    const ups_pose *__restrict__ base, GridArgs g,
                                                    ups_pose *__restrict__ best, int *__restrict__ best_score) {
    __shared__ int bs[256], bc[256];
    const int k = blockIdx.x, tid = threadIdx.x;
    int s = -1, ci = 0;
    for (int c = tid; c < C; c += 256) {
        const int v = scores[k * C + c];
        if (v > s) {
            s = v;
            ci = c;
        }
    }
    bs[tid] = s;
    bc[tid] = ci;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            const int s2 = bs[tid + w], c2 = bc[tid + w];
            if (s2 > bs[tid] || (s2 == bs[tid] && c2 < bc[tid])) {
                bs[tid] = s2;
                bc[tid] = c2;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        double R[9], t[3];
        candidate_pose(base[k], g, bc[0], R, t);
        for (int q = 0; q < 9; q++) best[k].R[q] = R[q];
        for (int q = 0; q < 3; q++) best[k].t[q] = t[q];
        if (best_score) best_score[k] = bs[0];
    }
}

ups_status launch_grid_search(const Inst *insts, const int *tile_start_l, int n, int K, int tiles,
                              const ups_pose *base, const GridArgs &g, int *scores, ups_pose *best, int *best_score,
                              hipStream_t s) {
    const int total = n * g.C;
    hipLaunchKernelGGL(k_grid_zero, dim3((total + 255) / 256), dim3(256), 0, s, scores, total);
    UPS_CHECK_HIP(hipGetLastError());
    if (tiles > 0) {
        // yaws per block: as many as keep 36 or fewer candidates per block
#define UPS_GRID_CASE(NXY, YB)                                                                              \
    case NXY:                                                                                               \
        hipLaunchKernelGGL((k_grid_score_yaw<NXY, YB>), dim3((g.n_yaw + YB - 1) / YB, tiles), dim3(kBlock), 0, s, \
                           insts, tile_start_l, n, K, base, g, scores);                                      \
        break;
        switch (g.n_xy) {
            UPS_GRID_CASE(1, 8)
            UPS_GRID_CASE(2, 4)
            UPS_GRID_CASE(3, 2)
            UPS_GRID_CASE(4, 1)
            UPS_GRID_CASE(5, 1)
            default:
                hipLaunchKernelGGL(k_grid_score, dim3(tiles, g.C), dim3(kBlock), 0, s, insts, tile_start_l, n, K,
                                   base, g, scores);
        }
#undef UPS_GRID_CASE
        UPS_CHECK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_grid_best, dim3(n), dim3(256), 0, s, g.C, scores, base, g, best, best_score);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
