// Instantiations and launchers of the persistent batch scheduler
// (k_sched_init, k_icp_persistent): pixels per thread 1 .. 64, the three
// precision modes, and the IRLS objective in the default precision mode.
#include <algorithm>

#include "ups_icp_kernels.hpp"

namespace ups {

// One block of 1024 threads: the first job of every registration taking part
// (mask null: all) that has iterations, its tiles under consecutive tickets in
// registration order, and the counters of the call (a new epoch).
__global__ __launch_bounds__(1024) void k_sched_init(SchedArgs A) {
    __shared__ int sc[2][2][1024];
    __shared__ int carry[2];
    __shared__ unsigned epoch;
    const int tid = threadIdx.x;
    if (tid == 0) {
        epoch = A.sched->epoch + 1u;
        carry[0] = carry[1] = 0;
    }
    __syncthreads();
    for (int c0 = 0; c0 < A.n; c0 += 1024) {
        const int k = c0 + tid;
        int v[2] = {0, 0};  // tiles, participation
        if (k < A.n) {
            if (!A.mask || A.mask[k]) {
                const SchedJob J = first_job(A, A.insts[k]);
                A.jobs[k] = J;
                if (J.mode == MODE_ITER) {  // else no iterations: only the evaluation, after this kernel
                    v[0] = J.ntiles;
                    v[1] = 1;
                }
            }
            A.arrived[k] = 0;
        }
        int buf = 0;
        sc[0][0][tid] = v[0];
        sc[0][1][tid] = v[1];
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            for (int q = 0; q < 2; q++)
                sc[buf ^ 1][q][tid] = sc[buf][q][tid] + (tid >= off ? sc[buf][q][tid - off] : 0);
            buf ^= 1;
            __syncthreads();
        }
        const int base = carry[0] + sc[buf][0][tid] - v[0];
        const unsigned long long tag = v[0] > 0 ? sched_tag(epoch, k, A.jobs[k]) : 0ull;
        for (int i = 0; i < v[0]; i++)
            if (base + i < A.map_size) A.tile_map[base + i] = tag | (unsigned)i;
        __syncthreads();
        if (tid < 2) carry[tid] += sc[buf][tid][1023];
        __syncthreads();
    }
    if (tid == 0) {
        Sched S;
        memset(&S, 0, sizeof(S));
        S.published = (unsigned)carry[0];
        S.outstanding = carry[1];
        S.error = carry[0] > A.map_size ? 1 : 0;
        S.epoch = epoch;
        *A.sched = S;
    }
}

namespace {

template <int K, int PREC, bool IRLS>
const void *persistent_fn() {
    return (const void *)&k_icp_persistent<K, PREC, IRLS>;
}

template <int K, int PREC>
const void *pick_fn(bool irls) {
    if constexpr (PREC == UPS_PREC_KAHAN_F64) {
        if (irls) return persistent_fn<K, PREC, true>();
    }
    return persistent_fn<K, PREC, false>();
}

const void *kernel_of(int K, int prec, bool irls) {
    const void *f = nullptr;
    auto pick = [&](auto kc, auto pc) { f = pick_fn<decltype(kc)::value, decltype(pc)::value>(irls); };
#define UPS_SCHED_P(KV)                                                                                  \
    if (prec == UPS_PREC_KAHAN_F64) pick(std::integral_constant<int, KV>{},                              \
                                         std::integral_constant<int, UPS_PREC_KAHAN_F64>{});             \
    if (prec == UPS_PREC_F32) pick(std::integral_constant<int, KV>{}, std::integral_constant<int, UPS_PREC_F32>{}); \
    if (prec == UPS_PREC_F64) pick(std::integral_constant<int, KV>{}, std::integral_constant<int, UPS_PREC_F64>{});
    switch (K) {
        case 1: UPS_SCHED_P(1) break;
        case 2: UPS_SCHED_P(2) break;
        case 4: UPS_SCHED_P(4) break;
        case 8: UPS_SCHED_P(8) break;
        case 16: UPS_SCHED_P(16) break;
        case 32: UPS_SCHED_P(32) break;
        case 64: UPS_SCHED_P(64) break;
        default: break;
    }
#undef UPS_SCHED_P
    return f;
}

}  // namespace

bool persistent_k_supported(int K) { return K >= 1 && K <= 64 && (K & (K - 1)) == 0; }

// Blocks per CU: the runtime's occupancy figure, or what the kernel's
// registers (512 per SIMD lane in granules of 8, one wavefront of the block
// per SIMD) and its LDS (160 KB per CU on gfx950) allow, whichever is larger.
// A launch may hold more blocks than fit at once: a block that has not
// started holds no ticket, and the others never wait for it.
int persistent_grid(int K, int prec, bool irls) {
    const void *f = kernel_of(K, prec, irls);
    if (!f) return 0;
    int per_cu = 0, dev = 0;
    hipDeviceProp_t prop;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBlock, 0) != hipSuccess || per_cu < 1) return 0;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, f) == hipSuccess && attr.numRegs > 0) {
        const int regs = (attr.numRegs + 7) / 8 * 8;
        const int by_regs = std::min(8, 512 / regs);
        const int by_lds = attr.sharedSizeBytes > 0 ? (int)((160 * 1024) / attr.sharedSizeBytes) : 8;
        per_cu = std::max(per_cu, std::min(by_regs, by_lds));
    }
    return per_cu * prop.multiProcessorCount;
}

ups_status launch_sched_init(const SchedArgs &A, hipStream_t s) {
    hipLaunchKernelGGL(k_sched_init, dim3(1), dim3(1024), 0, s, A);
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

ups_status launch_icp_persistent(int K, int prec, const SchedArgs &A, int blocks, hipStream_t s) {
    const void *f = kernel_of(K, prec, A.irls_delta > 0.f);
    if (!f) {
        set_error("no persistent kernel for this pixels-per-thread / precision");
        return UPS_ERR_INVALID_ARG;
    }
    const Inst *insts = A.insts;
    void *args[] = {(void *)&A, (void *)&insts};
    UPS_CHECK_HIP(hipLaunchKernel(f, dim3(blocks), dim3(kBlock), args, 0, s));
    return UPS_OK;
}

}  // namespace ups
