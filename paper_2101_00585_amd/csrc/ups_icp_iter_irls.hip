// Iteration / evaluation launches for the absolute-value objective of
// Equation 1 by iteratively reweighted least squares (single registrations,
// batches and batch subsets).  Instantiated for the default precision mode
// (Kahan-compensated FP32 sums, FP64 solve) only.
#include "ups_icp_kernels.hpp"

namespace ups {

static bool irls_precision_ok(int prec) {
    if (prec == UPS_PREC_KAHAN_F64) return true;
    set_error("the IRLS objective (irls_delta > 0) needs precision UPS_PREC_KAHAN_F64");
    return false;
}

template <int K>
static void launch_one_t(int mode, const Inst &I, const StepArgs &a0, int blocks, hipStream_t s) {
    const StepArgs a = with_tile_order(a0);
    constexpr int P = UPS_PREC_KAHAN_F64;
    if (mode == MODE_ITER)
        hipLaunchKernelGGL((k_icp_one<K, P, MODE_ITER, false, true>), dim3(blocks), dim3(kBlock), 0, s, I, a);
    else
        hipLaunchKernelGGL((k_icp_one<K, P, MODE_EVAL, false, true>), dim3(blocks), dim3(kBlock), 0, s, I, a);
}

ups_status launch_icp_one_irls(int K, int prec, int mode, const Inst &I, const StepArgs &a, int blocks,
                               hipStream_t s) {
    if (!irls_precision_ok(prec)) return UPS_ERR_INVALID_ARG;
    UPS_DISPATCH_K(K, launch_one_t<KK>(mode, I, a, blocks, s))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

template <int K, bool FUSED>
static void launch_batch_t(int mode, const Inst *insts, const int *tile_start, int n, const StepArgs &a0, int blocks,
                           hipStream_t s) {
    const StepArgs a = with_tile_order(a0);
    constexpr int P = UPS_PREC_KAHAN_F64;
    if (mode == MODE_ITER)
        hipLaunchKernelGGL((k_icp_batch<K, P, MODE_ITER, true, FUSED>), dim3(blocks), dim3(kBlock), 0, s, insts,
                           tile_start, n, a);
    else
        hipLaunchKernelGGL((k_icp_batch<K, P, MODE_EVAL, true, FUSED>), dim3(blocks), dim3(kBlock), 0, s, insts,
                           tile_start, n, a);
}

ups_status launch_icp_batch_irls(int K, int prec, int mode, const Inst *insts, const int *tile_start, int n,
                                 const StepArgs &a, int blocks, hipStream_t s, bool fused) {
    if (!irls_precision_ok(prec)) return UPS_ERR_INVALID_ARG;
    if (fused) {
        UPS_DISPATCH_K(K, (launch_batch_t<KK, true>(mode, insts, tile_start, n, a, blocks, s)))
    } else {
        UPS_DISPATCH_K(K, (launch_batch_t<KK, false>(mode, insts, tile_start, n, a, blocks, s)))
    }
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

template <int K>
static void launch_list_t(int mode, const Inst *insts, const Compact *hdr, const int *list, const int *start_l,
                          const StepArgs &a0, int blocks, hipStream_t s) {
    const StepArgs a = with_tile_order(a0);
    constexpr int P = UPS_PREC_KAHAN_F64;
    if (mode == MODE_ITER)
        hipLaunchKernelGGL((k_icp_batch_list<K, P, MODE_ITER, true>), dim3(blocks), dim3(kBlock), 0, s, insts, hdr,
                           list, start_l, a);
    else
        hipLaunchKernelGGL((k_icp_batch_list<K, P, MODE_EVAL, true>), dim3(blocks), dim3(kBlock), 0, s, insts, hdr,
                           list, start_l, a);
}

ups_status launch_icp_batch_list_irls(int K, int prec, int mode, const Inst *insts, const Compact *hdr,
                                      const int *list, const int *start_l, int n, const StepArgs &a, int blocks,
                                      hipStream_t s) {
    (void)n;
    if (!irls_precision_ok(prec)) return UPS_ERR_INVALID_ARG;
    UPS_DISPATCH_K(K, launch_list_t<KK>(mode, insts, hdr, list, start_l, a, blocks, s))
    UPS_CHECK_HIP(hipGetLastError());
    return UPS_OK;
}

}  // namespace ups
