// meso_kernels_fast.hip -- state-update kernels of the FP32-bulk /
// FP64-accumulate and pure FP32 modes.  Built with floating-point contraction
// (fused multiply-adds), which the FP64 mode's translation unit forbids.

#include "meso_device.h"

namespace meso {

template <class S, class R, int LIM>
static void launch_fast_t(const Desc &d, int mode, int final_pass, int src, hipStream_t st) {
    const dim3 grid(d.nstrips, d.nsegs), block(kThreads);
    switch (mode) {
        case kXY: hipLaunchKernelGGL((step_kernel<S, R, true, LIM, kXY, true>), grid, block, 0, st, d, src); break;
        case kYX: hipLaunchKernelGGL((step_kernel<S, R, true, LIM, kYX, true>), grid, block, 0, st, d, src); break;
        case kX:
            if (final_pass) hipLaunchKernelGGL((step_kernel<S, R, true, LIM, kX, true>), grid, block, 0, st, d, src);
            else hipLaunchKernelGGL((step_kernel<S, R, true, LIM, kX, false>), grid, block, 0, st, d, src);
            break;
        default:
            if (final_pass) hipLaunchKernelGGL((step_kernel<S, R, true, LIM, kY, true>), grid, block, 0, st, d, src);
            else hipLaunchKernelGGL((step_kernel<S, R, true, LIM, kY, false>), grid, block, 0, st, d, src);
            break;
    }
}

hipError_t launch_step_fast(const Desc &d, int prec, int lim, int mode, int final_pass, int src,
                            hipStream_t st) {
    if (prec == kPMix) {
        if (lim == 1) launch_fast_t<double, float, 1>(d, mode, final_pass, src, st);
        else launch_fast_t<double, float, 0>(d, mode, final_pass, src, st);
    } else {
        if (lim == 1) launch_fast_t<float, float, 1>(d, mode, final_pass, src, st);
        else launch_fast_t<float, float, 0>(d, mode, final_pass, src, st);
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
