// meso_kernels_fast.hip -- state-update kernels of the FP32-bulk /
// FP64-accumulate and pure FP32 modes.  Built with floating-point contraction
// (fused multiply-adds), which the FP64 mode's translation unit forbids.

#include "meso_device.h"

namespace meso {

hipError_t launch_step_fast(const Desc &d, int prec, int lim, int mode, int final_pass, int src,
                            hipStream_t st) {
    if (prec == kPMix) {
        if (lim == 1) launch_step_variants<double, float, true, 1, 6>(d, mode, final_pass, src, st);
        else launch_step_variants<double, float, true, 0, 6>(d, mode, final_pass, src, st);
    } else {
        if (lim == 1) launch_step_variants<float, float, true, 1, 6>(d, mode, final_pass, src, st);
        else launch_step_variants<float, float, true, 0, 6>(d, mode, final_pass, src, st);
    }
    return hipGetLastError();
}

template <class S, class R>
static void batched_fast_t(const Desc *descs, const int4 *tiles, int ntiles, int lim,
                           hipStream_t st) {
    if (lim == 1)
        hipLaunchKernelGGL((batched_step_kernel<S, R, true, 1>), dim3(ntiles), dim3(kThreads), 0,
                           st, descs, tiles);
    else
        hipLaunchKernelGGL((batched_step_kernel<S, R, true, 0>), dim3(ntiles), dim3(kThreads), 0,
                           st, descs, tiles);
}

hipError_t launch_batched_step_fast(const Desc *descs, const int4 *tiles, int ntiles, int prec,
                                    int lim, hipStream_t st) {
    if (prec == kPMix) batched_fast_t<double, float>(descs, tiles, ntiles, lim, st);
    else batched_fast_t<float, float>(descs, tiles, ntiles, lim, st);
    return hipGetLastError();
}

}  // namespace meso
