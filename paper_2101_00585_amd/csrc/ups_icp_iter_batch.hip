// Iteration / evaluation launches of a batch over all registrations (the pose
// in state slot 0), squared objective; the fused main-loop launches and the
// IRLS objective are handed to their own translation units.
#include "ups_icp_kernels.hpp"

namespace ups {

template <int K, int PREC>
static void launch_batch_t(int mode, const Inst *insts, const int *tile_start, int n, const StepArgs &a0, int blocks,
                           hipStream_t s) {
    const StepArgs a = with_tile_order(a0);
    if (mode == MODE_ITER)
        hipLaunchKernelGGL((k_icp_batch<K, PREC, MODE_ITER, false, false>), dim3(blocks), dim3(kBlock), 0, s, insts,
                           tile_start, n, a);
    else
        hipLaunchKernelGGL((k_icp_batch<K, PREC, MODE_EVAL, false, false>), dim3(blocks), dim3(kBlock), 0, s, insts,
                           tile_start, n, a);
}

ups_status launch_icp_batch(int K, int prec, int mode, const Inst *insts, const int *tile_start, int n,
                            const StepArgs &a, int blocks, hipStream_t s, bool fused) {
    if (a.irls_delta > 0.f) return launch_icp_batch_irls(K, prec, mode, insts, tile_start, n, a, blocks, s, fused);
    if (fused) return launch_icp_batch_fused(K, prec, mode, insts, tile_start, n, a, blocks, s);
    UPS_DISPATCH_P(prec, UPS_DISPATCH_K(K, launch_batch_t<KK, PP>(mode, insts, tile_start, n, a, blocks, s)))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
