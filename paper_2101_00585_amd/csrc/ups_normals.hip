// Surface normals of a panoramic range image (UPSLAM Section III-A): a rough
// normal from the cross product of the vectors to two image neighbours, then
// an edge-aware a-trous wavelet filter over LDS-staged tiles.
#include "ups_internal.hpp"

namespace ups {

// One thread per pixel.  The right neighbour wraps in azimuth; the lower
// neighbour is the previous row on the last row.  Rows of a wavefront share
// cache lines, so the neighbour reads are served from L1/L2.
__global__ __launch_bounds__(kBlock) void k_normals_raw(DGeom g, const float *__restrict__ depth,
                                                        float4 *__restrict__ out, float max_rel_jump) {
    const int npix = g.rows * g.cols;
    const int p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= npix) return;
    const int i = p / g.cols, j = p - i * g.cols;
    const float rc = depth[p];
    float4 o = make_float4(0.f, 0.f, 0.f, range_ok(g, rc) ? rc : 0.f);
    const int ja = (j + 1 == g.cols) ? 0 : j + 1;
    const int ib = (i + 1 < g.rows) ? i + 1 : i - 1;
    if (range_ok(g, rc) && ib >= 0) {
        const float ra = depth[i * g.cols + ja], rb = depth[ib * g.cols + j];
        if (range_ok(g, ra) && range_ok(g, rb) && !(fabsf(ra - rc) > max_rel_jump * rc) &&
            !(fabsf(rb - rc) > max_rel_jump * rc)) {
            const float3 uc = ray(g, i, j), ua = ray(g, i, ja), ub = ray(g, ib, j);
            const float3 pc = make_float3(rc * uc.x, rc * uc.y, rc * uc.z);
            const float3 a = make_float3(ra * ua.x - pc.x, ra * ua.y - pc.y, ra * ua.z - pc.z);
            const float3 b = make_float3(rb * ub.x - pc.x, rb * ub.y - pc.y, rb * ub.z - pc.z);
            const float3 n = cross3(a, b);
            const float nn = sqrtf(dot3(n, n));
            if (nn > 1e-6f * sqrtf(dot3(a, a)) * sqrtf(dot3(b, b))) {
                const float s = (dot3(n, pc) > 0.f) ? -1.f / nn : 1.f / nn;
                o.x = n.x * s;
                o.y = n.y * s;
                o.z = n.z * s;
            }
        }
    }
    out[p] = o;
}

constexpr int kTileW = 64, kTileH = 16;

// One a-trous level with taps spaced `step`: the block stages a
// (16 + 4 step) x (64 + 4 step) surfel tile (rows outside the image marked
// empty, columns wrapped) in LDS, then each thread filters 4 pixels of one
// column.  All edge-stopping factors of a tap share one exponential.
__global__ __launch_bounds__(kBlock) void k_atrous(DGeom g, const float4 *__restrict__ in, float4 *__restrict__ out,
                                                   int step, float inv_sigma_r, float inv_sigma_n2) {
    extern __shared__ float4 tile[];
    const int halo = 2 * step;
    const int LW = kTileW + 2 * halo, LH = kTileH + 2 * halo;
    const int x0 = blockIdx.x * kTileW, y0 = blockIdx.y * kTileH;
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
    const float h[5] = {1.f / 16, 4.f / 16, 6.f / 16, 4.f / 16, 1.f / 16};
    const int tx = threadIdx.x & (kTileW - 1), ty = threadIdx.x / kTileW;
#pragma unroll
    for (int k = 0; k < kTileH / (kBlock / kTileW); k++) {
        const int ly = ty + k * (kBlock / kTileW);
        const int gy = y0 + ly;
        if (gy >= g.rows) break;
        const float4 c = tile[(ly + halo) * LW + tx + halo];
        float4 o = make_float4(0.f, 0.f, 0.f, c.w);
        if (normal_ok(c)) {
            const float inv_rp = inv_sigma_r / c.w;
            float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll
            for (int dy = 0; dy < 5; dy++) {
                const float4 *row = tile + (ly + dy * step) * LW + tx;
#pragma unroll
                for (int dx = 0; dx < 5; dx++) {
                    const float4 q = row[dx * step];
                    if (!normal_ok(q)) continue;
                    const float dr = (q.w - c.w) * inv_rp;
                    const float dn = 2.f - 2.f * (c.x * q.x + c.y * q.y + c.z * q.z);
                    const float w = h[dy] * h[dx] * __expf(-(dr * dr + dn * inv_sigma_n2));
                    ax += w * q.x;
                    ay += w * q.y;
                    az += w * q.z;
                }
            }
            const float nn = sqrtf(ax * ax + ay * ay + az * az);
            if (nn > 0.f) {
                const float s = 1.f / nn;
                o.x = ax * s;
                o.y = ay * s;
                o.z = az * s;
            }
        }
        out[gy * g.cols + x0 + tx] = o;
    }
}

ups_status launch_normals(ups_context *ctx, const DGeom &g, const float *depth, float4 *surfel,
                          const ups_normal_params &p, hipStream_t s) {
    const int npix = g.rows * g.cols;
    const int L = p.atrous_levels;
    float4 *bufs[2] = {surfel, ctx->tmp_surfel};
    // ping-pong so that the last level writes `surfel`
    float4 *raw = (L % 2 == 0) ? surfel : ctx->tmp_surfel;
    hipLaunchKernelGGL(k_normals_raw, dim3((npix + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g, depth, raw,
                       p.max_rel_jump);
    UPS_CHECK_HIP(hipGetLastError());
    const float4 *src = raw;
    for (int l = 0; l < L; l++) {
        float4 *dst = ((L - 1 - l) % 2 == 0) ? bufs[0] : bufs[1];
        const int step = 1 << l;
        const size_t lds = (size_t)(kTileW + 4 * step) * (kTileH + 4 * step) * sizeof(float4);
        dim3 grid(g.cols / kTileW, (g.rows + kTileH - 1) / kTileH);
        hipLaunchKernelGGL(k_atrous, grid, dim3(kBlock), lds, s, g, src, dst, step, 1.f / p.sigma_r,
                           1.f / (p.sigma_n * p.sigma_n));
        UPS_CHECK_HIP(hipGetLastError());
        src = dst;
    }
    return UPS_OK;
}

}  // namespace ups
