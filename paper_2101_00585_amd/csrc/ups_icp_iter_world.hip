// Iteration / evaluation launches of the world-frame variant of a single
// registration (FP32 world coordinates; the precision study).
#include "ups_icp_kernels.hpp"

namespace ups {

template <int K, int PREC>
static void launch_t(int mode, const Inst &I, const StepArgs &a0, int blocks, hipStream_t s) {
    const StepArgs a = with_tile_order(a0);
    if (mode == MODE_ITER)
        hipLaunchKernelGGL((k_icp_one<K, PREC, MODE_ITER, true, false>), dim3(blocks), dim3(kBlock), 0, s, I, a);
    else
        hipLaunchKernelGGL((k_icp_one<K, PREC, MODE_EVAL, true, false>), dim3(blocks), dim3(kBlock), 0, s, I, a);
}

ups_status launch_icp_one_world(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                                hipStream_t s) {
    UPS_DISPATCH_P(prec, UPS_DISPATCH_K(K, launch_t<KK, PP>(mode, I, a, blocks, s)))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
