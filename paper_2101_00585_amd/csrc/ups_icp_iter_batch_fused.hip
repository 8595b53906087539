// Iteration / evaluation launches of a batch's main loop, squared objective:
// each block first applies its registration's pending update (the fused
// prologue), so the loop needs no separate solve launches.
#include "ups_icp_kernels.hpp"

namespace ups {

template <int K, int PREC>
static void launch_fused_t(int mode, const Inst *insts, const int *tile_start, int n, const StepArgs &a0, int blocks,
                           hipStream_t s) {
    const StepArgs a = with_tile_order(a0);
    if (mode == MODE_ITER)
        hipLaunchKernelGGL((k_icp_batch<K, PREC, MODE_ITER, false, true>), dim3(blocks), dim3(kBlock), 0, s, insts,
                           tile_start, n, a);
    else
        hipLaunchKernelGGL((k_icp_batch<K, PREC, MODE_EVAL, false, true>), dim3(blocks), dim3(kBlock), 0, s, insts,
                           tile_start, n, a);
}

ups_status launch_icp_batch_fused(int K, int prec, int mode, const Inst *insts, const int *tile_start, int n,
                                  const StepArgs &a, int blocks, hipStream_t s) {
    UPS_DISPATCH_P(prec, UPS_DISPATCH_K(K, launch_fused_t<KK, PP>(mode, insts, tile_start, n, a, blocks, s)))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
