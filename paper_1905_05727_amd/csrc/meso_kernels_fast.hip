// meso_kernels_fast.hip -- state-update kernels of the FP32-bulk /
// FP64-accumulate mode (inert liquids).  Built with floating-point
// contraction (fused multiply-adds), which the FP64 mode's translation unit
// forbids.

#include "meso_device.h"

namespace meso {

hipError_t launch_step_fast(const Desc &d, int lim, int mode, int final_pass, int src,
                            hipStream_t st) {
    if (lim == 1) launch_step_variants<double, float, true, 1, 6>(d, mode, final_pass, src, st);
    else launch_step_variants<double, float, true, 0, 6>(d, mode, final_pass, src, st);
    return hipGetLastError();
}

hipError_t launch_batched_step_fast(const Desc *descs, const int4 *tiles, int ntiles, int lim,
                                    int eos, hipStream_t st) {
    launch_batched_variants<double, float, true, 6>(descs, tiles, ntiles, lim, eos, st);
    return hipGetLastError();
}

}  // namespace meso
