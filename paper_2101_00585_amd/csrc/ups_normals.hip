// Surface normals of a panoramic range image (UPSLAM Section III-A): a rough
// normal from the cross product of the vectors to two image neighbours, then
// an edge-aware a-trous wavelet filter over LDS-staged tiles.
#include "ups_internal.hpp"

namespace ups {

// Raw normal of pixel (i, j) from its range rc and the ranges of its right
// neighbour (i, j+1 mod cols) and lower neighbour (i+1, j) -- (i-1, j) on the
// last row: the normalised cross product of the two difference vectors,
// oriented towards the sensor; zero when a range is invalid, a neighbour jumps
// by more than max_rel_jump * rc, or the cross product is degenerate.
// The same from the rays of the three pixels (uc: the pixel, ua: its right
// neighbour, ub: the lower one); ib < 0 means the lower neighbour is missing.
__device__ __forceinline__ float3 raw_normal_rays(const DGeom &g, int ib, float rc, float ra, float rb, float3 uc,
                                                  float3 ua, float3 ub, float max_rel_jump) {
    float3 o = make_float3(0.f, 0.f, 0.f);
    if (!(range_ok(g, rc) && ib >= 0 && range_ok(g, ra) && range_ok(g, rb))) return o;
    if (fabsf(ra - rc) > max_rel_jump * rc || fabsf(rb - rc) > max_rel_jump * rc) return o;
    const float3 pc = make_float3(rc * uc.x, rc * uc.y, rc * uc.z);
    const float3 a = make_float3(ra * ua.x - pc.x, ra * ua.y - pc.y, ra * ua.z - pc.z);
    const float3 b = make_float3(rb * ub.x - pc.x, rb * ub.y - pc.y, rb * ub.z - pc.z);
    const float3 n = cross3(a, b);
    const float nn = __builtin_amdgcn_sqrtf(dot3(n, n));
    if (!(nn > 1e-6f * __builtin_amdgcn_sqrtf(dot3(a, a) * dot3(b, b)))) return o;
    const float inv = __builtin_amdgcn_rcpf(nn);
    const float s = (dot3(n, pc) > 0.f) ? -inv : inv;
    return make_float3(n.x * s, n.y * s, n.z * s);
}

__device__ __forceinline__ float3 raw_normal(const DGeom &g, int i, int j, int ib, float rc, float ra, float rb,
                                             float max_rel_jump) {
    if (!(range_ok(g, rc) && ib >= 0 && range_ok(g, ra) && range_ok(g, rb))) return make_float3(0.f, 0.f, 0.f);
    const int ja = (j + 1 == g.cols) ? 0 : j + 1;
    return raw_normal_rays(g, ib, rc, ra, rb, ray(g, i, j), ray(g, i, ja), ray(g, ib, j), max_rel_jump);
}

// Ray of a pixel from its row's (cos el, sin el) and its column's (cos az, sin az).
__device__ __forceinline__ float3 ray_of(float2 e, float2 a) { return make_float3(e.x * a.x, e.x * a.y, e.y); }

// Raw normals only (no smoothing): one thread per pixel; the neighbour reads
// are served from L1/L2.
__global__ __launch_bounds__(kBlock) void k_normals_raw(DGeom g, const float *__restrict__ depth,
                                                        float4 *__restrict__ out, float max_rel_jump) {
    const int npix = g.rows * g.cols;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const int i = p / g.cols, j = p - i * g.cols;
    const float rc = depth[p];
    const int ja = (j + 1 == g.cols) ? 0 : j + 1;
    const int ib = (i + 1 < g.rows) ? i + 1 : i - 1;
    const float ra = depth[i * g.cols + ja], rb = ib >= 0 ? depth[ib * g.cols + j] : 0.f;
    const float3 n = raw_normal(g, i, j, ib, rc, ra, rb, max_rel_jump);
    out[p] = make_float4(n.x, n.y, n.z, range_ok(g, rc) ? rc : 0.f);
}

// Output tiles of the a-trous passes: 64 pixels wide, TH rows high, TH / 4
// rows per thread.  Batches use 16 rows (the halo of recomputed raw normals
// and of staged neighbours shrinks with the tile's height); a single panorama
// uses 4 rows, which gives it enough workgroups to fill the GPU.
constexpr int kTileW = 64, kTileHBatch = 16, kTileHOne = 4;

// One a-trous output from an LDS surfel tile of row pitch LW whose pixel
// (ly, lx) is the output (ly + 2 step, lx + 2 step) of the tile: 5x5 B3-spline
// taps spaced `step`, weight h[dy] h[dx] exp(-(dr^2 + (2 - 2 n_p.n_q)/sigma_n^2))
// with dr = (r_q - r_p)/(sigma_r r_p), renormalised; the range is unchanged.
// The whole weight is one exp2: log2 e and 1/sigma_n^2 are folded into a
// scaled copy of the centre normal, sqrt(log2 e)/(sigma_r r_p) into the range
// difference and log2(h[dy] h[dx]) into the exponent, so a tap costs three
// FMAs for the normal term, two for the range term and three to accumulate.
// Taps without a normal need no test: their zero normal adds nothing to the
// weighted sum, and the sum is renormalised rather than divided by the total
// weight.
__device__ __forceinline__ float4 atrous_tap_sum(const float4 *tile, int LW, int ly, int lx, int step,
                                                 float inv_sigma_r, float inv_sigma_n2) {
    constexpr float kLog2e = 1.4426950408889634f;
    // log2 of h = (1, 4, 6, 4, 1) / 16
    constexpr float lh[5] = {-4.f, -2.f, -1.4150374992788437f, -2.f, -4.f};
    const float4 c = tile[(ly + 2 * step) * LW + lx + 2 * step];
    float4 o = make_float4(0.f, 0.f, 0.f, c.w);
    if (!normal_ok(c)) return o;
    // log2 e (2 - 2 n_p.n_q) / sigma_n^2 = kn - kn n_p.n_q
    const float kn = 2.f * kLog2e * inv_sigma_n2;
    const float cx = kn * c.x, cy = kn * c.y, cz = kn * c.z;
    // log2 e ((r_q - r_p) / (sigma_r r_p))^2 = (r_q sr - r_p sr)^2
    const float sr = 1.2011224087864498f * inv_sigma_r * __builtin_amdgcn_rcpf(c.w);  // sqrt(log2 e) / (sigma_r r_p)
    const float csr = -c.w * sr;
    float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
    for (int dy = 0; dy < 5; dy++) {
        const float4 *row = tile + (ly + dy * step) * LW + lx;
#pragma unroll
        for (int dx = 0; dx < 5; dx++) {
            const float4 q = row[dx * step];
            float e = fmaf(cx, q.x, lh[dy] + lh[dx] - kn);
            e = fmaf(cy, q.y, e);
            e = fmaf(cz, q.z, e);
            const float d = fmaf(q.w, sr, csr);
            e = fmaf(-d, d, e);
            const float w = __builtin_amdgcn_exp2f(e);
            ax = fmaf(w, q.x, ax);
            ay = fmaf(w, q.y, ay);
            az = fmaf(w, q.z, az);
        }
    }
    const float nn2 = ax * ax + ay * ay + az * az;
    if (nn2 > 0.f) {
        const float s = __builtin_amdgcn_rsqf(nn2);
        o.x = ax * s;
        o.y = ay * s;
        o.z = az * s;
    }
    return o;
}

// Pyramid levels 1-3 of an image from its level-0 pixel (i, j): level-l pixel
// (i >> l, j >> l) when i and j are multiples of 2^l (every 2^l-th row and
// column; pyr[l - 1] null past the last level).
__device__ __forceinline__ void store_pyramid(const DGeom &g, float4 *const *pyr, int i, int j, float4 v) {
#pragma unroll
    for (int l = 1; l <= 3; l++) {
        float4 *dst = pyr[l - 1];
        if (dst && ((i | j) & ((1 << l) - 1)) == 0) dst[(i >> l) * (g.cols >> l) + (j >> l)] = v;
    }
}

// One a-trous level with taps spaced STEP for the kTileH x 64 output tile at
// (x0, y0): the block stages the (kTileH + 4 STEP) x (64 + 4 STEP) surfel
// tile around it in LDS (rows outside the image empty, columns wrapped), one
// output row per wavefront and pass.  STEP is a template parameter so that
// the staging loop divides by a constant and every tap reads LDS at a
// constant offset from the output's address.
template <int kTileH, int STEP>
__device__ __forceinline__ void atrous_tile(const DGeom &g, const float4 *__restrict__ in, float4 *__restrict__ out,
                                            int x0, int y0, float inv_sigma_r, float inv_sigma_n2, float4 *tile,
                                            float4 *const *pyr) {
    constexpr int halo = 2 * STEP;
    constexpr int LW = kTileW + 2 * halo, LH = kTileH + 2 * halo;
    for (int idx = threadIdx.x; idx < LW * LH; idx += kBlock) {
        const int ly = idx / LW, lx = idx - ly * LW;
        const int gy = y0 - halo + ly;
        int gx = x0 - halo + lx;
        gx = gx < 0 ? gx + g.cols : (gx >= g.cols ? gx - g.cols : gx);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gy >= 0 && gy < g.rows) v = in[gy * g.cols + gx];
        tile[idx] = v;
    }
    __syncthreads();
    const int tx = threadIdx.x & (kTileW - 1);
    for (int ty = threadIdx.x / kTileW; ty < kTileH; ty += kBlock / kTileW) {
        const int gy = y0 + ty;
        if (gy >= g.rows) break;
        const float4 v = atrous_tap_sum(tile, LW, ty, tx, STEP, inv_sigma_r, inv_sigma_n2);
        out[gy * g.cols + x0 + tx] = v;
        if (pyr) store_pyramid(g, pyr, gy, x0 + tx, v);
    }
}

template <int kTileH, int STEP>
constexpr int atrous_tile_elems() { return (kTileW + 4 * STEP) * (kTileH + 4 * STEP); }

template <int STEP>
__global__ __launch_bounds__(kBlock) void k_atrous(DGeom g, const float4 *__restrict__ in, float4 *__restrict__ out,
                                                   float inv_sigma_r, float inv_sigma_n2) {
    __shared__ float4 tile[atrous_tile_elems<kTileHOne, STEP>()];
    atrous_tile<kTileHOne, STEP>(g, in, out, blockIdx.x * kTileW, blockIdx.y * kTileHOne, inv_sigma_r, inv_sigma_n2,
                                 tile, nullptr);
}

// Raw normals and the first a-trous level (step 1) in one pass: the block
// stages the ranges of its 16 x 64 outputs plus a 2-pixel halo (and the
// neighbour row/column the cross products need), computes the raw normals of
// the 20 x 68 halo tile into LDS, then filters.
template <int kTileH>
__device__ __forceinline__ void normals_atrous_tile(const DGeom &g, const float *__restrict__ depth,
                                                    float4 *__restrict__ out, int x0, int y0, float max_rel_jump,
                                                    float inv_sigma_r, float inv_sigma_n2, float4 *const *pyr) {
    constexpr int kFH = kTileH + 4, kFW = kTileW + 4;  // raw-normal tile
    constexpr int kDH = kFH + 2, kDW = kFW + 1;        // range tile: one row above and below, one column right
    static_assert(kDH + kDW <= kBlock, "ray tables of the tile: one entry per thread");
    __shared__ float rng[kDH][kDW];
    __shared__ float2 lrow[kDH], lcol[kDW];  // ray tables of the range tile's rows and columns
    __shared__ float4 raw[kFH * kFW];
    if (threadIdx.x < kDH) {
        const int gy = y0 - 3 + (int)threadIdx.x;
        lrow[threadIdx.x] = (gy >= 0 && gy < g.rows) ? ldg(g.lut_row, gy * g.stride) : make_float2(0.f, 0.f);
    } else if (threadIdx.x < kDH + kDW) {
        const int lx = threadIdx.x - kDH;
        int gx = x0 - 2 + lx;
        gx = gx < 0 ? gx + g.cols : (gx >= g.cols ? gx - g.cols : gx);
        lcol[lx] = ldg(g.lut_col, gx * g.stride);
    }
    // ranges of rows y0-3 .. y0+kTileH+2 and columns x0-2 .. x0+kTileW+2
    for (int idx = threadIdx.x; idx < kDH * kDW; idx += kBlock) {
        const int ly = idx / kDW, lx = idx - ly * kDW;
        const int gy = y0 - 3 + ly;
        int gx = x0 - 2 + lx;
        gx = gx < 0 ? gx + g.cols : (gx >= g.cols ? gx - g.cols : gx);
        rng[ly][lx] = (gy >= 0 && gy < g.rows) ? depth[gy * g.cols + gx] : 0.f;
    }
    __syncthreads();
    // raw normals of rows y0-2 .. y0+kTileH+1, columns x0-2 .. x0+kTileW+1
    for (int idx = threadIdx.x; idx < kFH * kFW; idx += kBlock) {
        const int ly = idx / kFW, lx = idx - ly * kFW;
        const int gy = y0 - 2 + ly;
        int gx = x0 - 2 + lx;
        gx = gx < 0 ? gx + g.cols : (gx >= g.cols ? gx - g.cols : gx);
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gy >= 0 && gy < g.rows) {
            const int dy = ly + 1, dx = lx;  // this pixel in the range tile
            const float rc = rng[dy][dx];
            const int ib = (gy + 1 < g.rows) ? gy + 1 : gy - 1;
            const int db = (ib == gy + 1) ? dy + 1 : dy - 1;  // the lower neighbour's row in the range tile
            const float3 n = raw_normal_rays(g, ib, rc, rng[dy][dx + 1], rng[db][dx], ray_of(lrow[dy], lcol[dx]),
                                             ray_of(lrow[dy], lcol[dx + 1]), ray_of(lrow[db], lcol[dx]),
                                             max_rel_jump);
            v = make_float4(n.x, n.y, n.z, range_ok(g, rc) ? rc : 0.f);
        }
        raw[idx] = v;
    }
    __syncthreads();
    const int tx = threadIdx.x & (kTileW - 1);
    for (int ty = threadIdx.x / kTileW; ty < kTileH; ty += kBlock / kTileW) {
        const int gy = y0 + ty;
        if (gy >= g.rows) break;
        const float4 v = atrous_tap_sum(raw, kFW, ty, tx, 1, inv_sigma_r, inv_sigma_n2);
        out[gy * g.cols + x0 + tx] = v;
        if (pyr) store_pyramid(g, pyr, gy, x0 + tx, v);
    }
}

__global__ __launch_bounds__(kBlock) void k_normals_atrous(DGeom g, const float *__restrict__ depth,
                                                           float4 *__restrict__ out, float max_rel_jump,
                                                           float inv_sigma_r, float inv_sigma_n2) {
    normals_atrous_tile<kTileHOne>(g, depth, out, blockIdx.x * kTileW, blockIdx.y * kTileHOne, max_rel_jump,
                                   inv_sigma_r, inv_sigma_n2, nullptr);
}

// ---- batched: block -> (image, tile) from a table, one word per tile:
// (image << kNormTileBits) | tile of the image

__global__ __launch_bounds__(kBlock) void k_normals_atrous_batch(const NormImg *__restrict__ imgs,
                                                                 const unsigned *__restrict__ tile_of,
                                                                 int out_tmp, int write_pyr, float max_rel_jump,
                                                                 float inv_sigma_r, float inv_sigma_n2) {
    const unsigned v = tile_of[blockIdx.x];
    const NormImg &im = imgs[v >> kNormTileBits];
    const int t = (int)(v & ((1u << kNormTileBits) - 1)), tx = im.g.cols / kTileW;
    const int by = t / tx, bx = t - by * tx;
    normals_atrous_tile<kTileHBatch>(im.g, im.depth, out_tmp ? im.tmp : im.out, bx * kTileW, by * kTileHBatch,
                                     max_rel_jump, inv_sigma_r, inv_sigma_n2, write_pyr ? im.pyr : nullptr);
}

template <int STEP>
__global__ __launch_bounds__(kBlock) void k_atrous_batch(const NormImg *__restrict__ imgs,
                                                         const unsigned *__restrict__ tile_of, int src_tmp,
                                                         int write_pyr, float inv_sigma_r, float inv_sigma_n2) {
    __shared__ float4 tile[atrous_tile_elems<kTileHBatch, STEP>()];
    const unsigned v = tile_of[blockIdx.x];
    const NormImg &im = imgs[v >> kNormTileBits];
    const int t = (int)(v & ((1u << kNormTileBits) - 1)), tx = im.g.cols / kTileW;
    const int by = t / tx, bx = t - by * tx;
    atrous_tile<kTileHBatch, STEP>(im.g, src_tmp ? im.tmp : im.out, src_tmp ? im.out : im.tmp, bx * kTileW,
                                   by * kTileHBatch, inv_sigma_r, inv_sigma_n2, tile, write_pyr ? im.pyr : nullptr);
}

// Tiles of a panorama in the batched a-trous launches.
int normal_tiles(const DGeom &g) { return (g.cols / kTileW) * ((g.rows + kTileHBatch - 1) / kTileHBatch); }

ups_status launch_normals_batch(const NormImg *imgs, const unsigned *tile_of, int total_tiles,
                                const ups_normal_params &p, int write_pyr, hipStream_t s) {
    const int L = p.atrous_levels;
    const float inv_sr = 1.f / p.sigma_r, inv_sn2 = 1.f / (p.sigma_n * p.sigma_n);
    if (L == 0 || total_tiles == 0) {
        if (total_tiles > 0) {
            set_error("batched normals need at least one a-trous level");
            return UPS_ERR_UNSUPPORTED;
        }
        return UPS_OK;
    }
    // ping-pong between out and tmp so that the last level writes out
    int in_tmp = (L - 1) % 2;
    // the last pass writes the surfel images (and, with write_pyr, their pyramids)
    hipLaunchKernelGGL(k_normals_atrous_batch, dim3(total_tiles), dim3(kBlock), 0, s, imgs, tile_of, in_tmp,
                       (L == 1) ? write_pyr : 0, p.max_rel_jump, inv_sr, inv_sn2);
    UPS_CHECK_HIP(hipGetLastError());
    for (int l = 1; l < L; l++) {
        // levels 1 and 2 (taps spaced 2 and 4); the caller limits the levels to 3
        const int last = (l == L - 1) ? write_pyr : 0;
        if (l == 1)
            hipLaunchKernelGGL(k_atrous_batch<2>, dim3(total_tiles), dim3(kBlock), 0, s, imgs, tile_of, in_tmp,
                               last, inv_sr, inv_sn2);
        else
            hipLaunchKernelGGL(k_atrous_batch<4>, dim3(total_tiles), dim3(kBlock), 0, s, imgs, tile_of, in_tmp,
                               last, inv_sr, inv_sn2);
        UPS_CHECK_HIP(hipGetLastError());
        in_tmp ^= 1;
    }
    return UPS_OK;
}

ups_status launch_normals(ups_context *ctx, const DGeom &g, const float *depth, float4 *surfel,
                          const ups_normal_params &p, hipStream_t s) {
    const int npix = g.rows * g.cols;
    const int L = p.atrous_levels;
    const float inv_sr = 1.f / p.sigma_r, inv_sn2 = 1.f / (p.sigma_n * p.sigma_n);
    if (L == 0) {
        hipLaunchKernelGGL(k_normals_raw, dim3((npix + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g, depth, surfel,
                           p.max_rel_jump);
        UPS_CHECK_HIP(hipGetLastError());
        return UPS_OK;
    }
    const dim3 grid(g.cols / kTileW, (g.rows + kTileHOne - 1) / kTileHOne);
    // ping-pong so that the last level writes `surfel`
    float4 *bufs[2] = {surfel, ctx->tmp_surfel};
    float4 *dst = bufs[(L - 1) % 2];
    hipLaunchKernelGGL(k_normals_atrous, grid, dim3(kBlock), 0, s, g, depth, dst, p.max_rel_jump, inv_sr, inv_sn2);
    UPS_CHECK_HIP(hipGetLastError());
    const float4 *src = dst;
    for (int l = 1; l < L; l++) {
        dst = bufs[(L - 1 - l) % 2];
        // levels 1 and 2 (taps spaced 2 and 4); the caller limits the levels to 3
        if (l == 1) hipLaunchKernelGGL(k_atrous<2>, grid, dim3(kBlock), 0, s, g, src, dst, inv_sr, inv_sn2);
        else hipLaunchKernelGGL(k_atrous<4>, grid, dim3(kBlock), 0, s, g, src, dst, inv_sr, inv_sn2);
        UPS_CHECK_HIP(hipGetLastError());
        src = dst;
    }
    return UPS_OK;
}

}  // namespace ups
