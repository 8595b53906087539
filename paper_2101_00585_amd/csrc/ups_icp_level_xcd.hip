// The one-XCD level kernel of single registrations (k_icp_level_xcd): every
// precision mode, keyframe-frame and world-frame arithmetic, the IRLS
// objective in the default precision mode.
#include "ups_icp_kernels.hpp"

namespace ups {

template <int K, int PREC>
static void launch_level_t(const Inst &I, const StepArgs &a0, int iters, int blocks, hipStream_t s) {
    const StepArgs a = with_tile_order(a0);
    if (I.world)
        hipLaunchKernelGGL((k_icp_level_xcd<K, PREC, true, false>), dim3(blocks), dim3(kBlock), 0, s, I, a, iters, 0u);
    else if (a.irls_delta > 0.f) {
        if constexpr (PREC == UPS_PREC_KAHAN_F64)
            hipLaunchKernelGGL((k_icp_level_xcd<K, PREC, false, true>), dim3(blocks), dim3(kBlock), 0, s, I, a, iters,
                               0u);
    } else
        hipLaunchKernelGGL((k_icp_level_xcd<K, PREC, false, false>), dim3(blocks), dim3(kBlock), 0, s, I, a, iters,
                           0u);
}

ups_status launch_icp_level_xcd(int K, int prec, const Inst &I, const StepArgs &a, int iters, int tiles,
                                hipStream_t s) {
    if (!I.xsync || tiles > kLevelXcdMaxTiles || (a.irls_delta > 0.f && (I.world || prec != UPS_PREC_KAHAN_F64))) {
        set_error("no one-XCD level kernel for this registration");
        return UPS_ERR_INVALID_ARG;
    }
    // eight workgroups per tile: the XCD that takes the tiles receives one per tile
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
