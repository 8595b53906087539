// Iteration / evaluation launches of a single registration, squared
// objective, keyframe-frame arithmetic (the default path), and the one-XCD
// level kernel of single registrations (k_icp_level_xcd: every precision
// mode, keyframe-frame and world-frame arithmetic, the IRLS objective in the
// default precision mode).  Both are in the translation unit that holds the
// phase timestamps of the instrumented build.
#define UPS_PHASE_TU
#include <atomic>

#include "ups_icp_kernels.hpp"

#ifdef UPS_PHASE_TIMESTAMPS
namespace ups {
__device__ unsigned long long g_phase_mark[kPhaseLaunches][5];
__device__ unsigned long long g_phase_first[kPhaseLaunches];
__device__ unsigned long long g_phase_last[kPhaseLaunches];
}  // namespace ups

// Instrumented build only: copy the phase timestamps of the last calls to
// out[64 * 7] (per launch: the five marks of tile 0, the earliest entry, the
// latest exit), then reset them for the next call.
extern "C" ups_status ups_debug_phase_read(unsigned long long *out) {
    using namespace ups;
    static unsigned long long h[kPhaseLaunches * 7];
    unsigned long long *marks = h, *first = h + kPhaseLaunches * 5, *last = h + kPhaseLaunches * 6;
    UPS_CHECK_HIP(hipMemcpyFromSymbol(marks, HIP_SYMBOL(g_phase_mark), sizeof(g_phase_mark)));
    UPS_CHECK_HIP(hipMemcpyFromSymbol(first, HIP_SYMBOL(g_phase_first), sizeof(g_phase_first)));
    UPS_CHECK_HIP(hipMemcpyFromSymbol(last, HIP_SYMBOL(g_phase_last), sizeof(g_phase_last)));
    for (int i = 0; i < kPhaseLaunches * 7; i++) out[i] = h[i];
    unsigned long long lo[kPhaseLaunches], hi[kPhaseLaunches];
    for (int i = 0; i < kPhaseLaunches; i++) {
        lo[i] = ~0ull;
        hi[i] = 0;
    }
    UPS_CHECK_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_phase_first), lo, sizeof(lo)));
    UPS_CHECK_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_phase_last), hi, sizeof(hi)));
    return UPS_OK;
}
#endif

namespace ups {

template <int K, int PREC>
static void launch_t(int mode, const Inst &I, const StepArgs &a0, int blocks, hipStream_t s) {
    const StepArgs a = with_tile_order(a0);
    if (mode == MODE_ITER)
        hipLaunchKernelGGL((k_icp_one<K, PREC, MODE_ITER, false, false>), dim3(blocks), dim3(kBlock), 0, s, I, a);
    else
        hipLaunchKernelGGL((k_icp_one<K, PREC, MODE_EVAL, false, false>), dim3(blocks), dim3(kBlock), 0, s, I, a);
}

ups_status launch_icp_one_plain(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                                hipStream_t s) {
    UPS_DISPATCH_P(prec, UPS_DISPATCH_K(K, launch_t<KK, PP>(mode, I, a, blocks, s)))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

// The XCD whose workgroups take the tiles, rotated over the 8 from launch to
// launch (process-wide).
static std::atomic<unsigned> g_level_xcd{0};

template <int K, int PREC>
static void launch_level_t(const Inst &I, const StepArgs &a0, int iters, int blocks, hipStream_t s) {
    const StepArgs a = with_tile_order(a0);
    const unsigned spin = level_spin_limit();
    const unsigned xcd = g_level_xcd.fetch_add(1, std::memory_order_relaxed) & 7u;
    if (I.world)
        hipLaunchKernelGGL((k_icp_level_xcd<K, PREC, true, false>), dim3(blocks), dim3(kBlock), 0, s, I, a, iters, xcd,
                           0u, spin);
    else if (a.irls_delta > 0.f) {
        if constexpr (PREC == UPS_PREC_KAHAN_F64)
            hipLaunchKernelGGL((k_icp_level_xcd<K, PREC, false, true>), dim3(blocks), dim3(kBlock), 0, s, I, a, iters,
                               xcd, 0u, spin);
    } else
        hipLaunchKernelGGL((k_icp_level_xcd<K, PREC, false, false>), dim3(blocks), dim3(kBlock), 0, s, I, a, iters,
                           xcd, 0u, spin);
}

ups_status launch_icp_level_xcd(int K, int prec, const Inst &I, const StepArgs &a, int iters, int tiles,
                                hipStream_t s) {
    if (!I.xsync || tiles > kLevelXcdMaxTiles || (a.irls_delta > 0.f && (I.world || prec != UPS_PREC_KAHAN_F64))) {
        set_error("no one-XCD level kernel for this registration");
        return UPS_ERR_INVALID_ARG;
    }
    // eight workgroups per tile: each XCD, the one that takes the tiles among them, receives one per tile
    const int blocks = 8 * tiles;
    switch (K) {
        case 1: UPS_DISPATCH_P(prec, (launch_level_t<1, PP>(I, a, iters, blocks, s))) break;
        case 2: UPS_DISPATCH_P(prec, (launch_level_t<2, PP>(I, a, iters, blocks, s))) break;
        default: set_error("one-XCD level kernel: pixels per thread must be 1 or 2"); return UPS_ERR_INVALID_ARG;
    }
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
