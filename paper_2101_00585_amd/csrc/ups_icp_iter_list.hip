// Iteration / evaluation launches over the Compact list of a subset of a
// batch, squared objective.
#include "ups_icp_kernels.hpp"

namespace ups {

template <int K, int PREC>
static void launch_list_t(int mode, const Inst *insts, const Compact *hdr, const int *list, const int *start_l,
                          const StepArgs &a0, int blocks, hipStream_t s) {
    const StepArgs a = with_tile_order(a0);
    if (mode == MODE_ITER)
        hipLaunchKernelGGL((k_icp_batch_list<K, PREC, MODE_ITER, false>), dim3(blocks), dim3(kBlock), 0, s, insts,
                           hdr, list, start_l, a);
    else
        hipLaunchKernelGGL((k_icp_batch_list<K, PREC, MODE_EVAL, false>), dim3(blocks), dim3(kBlock), 0, s, insts,
                           hdr, list, start_l, a);
}

ups_status launch_icp_batch_list(int K, int prec, int mode, const Inst *insts, const Compact *hdr, const int *list,
                                 const int *start_l, int n, const StepArgs &a, int blocks, hipStream_t s) {
    if (blocks <= 0) return UPS_OK;
    if (a.irls_delta > 0.f)
        return launch_icp_batch_list_irls(K, prec, mode, insts, hdr, list, start_l, n, a, blocks, s);
    UPS_DISPATCH_P(prec, UPS_DISPATCH_K(K, launch_list_t<KK, PP>(mode, insts, hdr, list, start_l, a, blocks, s)))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
