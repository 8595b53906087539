// Iteration / evaluation launches of a single registration, squared
// objective, keyframe-frame arithmetic (the default path).
#define UPS_PHASE_TU
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

}  // namespace ups
