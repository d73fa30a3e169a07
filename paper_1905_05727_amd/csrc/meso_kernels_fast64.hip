// meso_kernels_fast64.hip -- state-update kernels of the fast FP64 mode: FP64
// state and arithmetic throughout, divisions and square roots from the
// hardware seeds refined by a second-order series, built with floating-point
// contraction (fused multiply-adds).  Inert and reactive liquids; the
// reactive fused kernel is held to two waves per SIMD like the FP64 one.

#define MESO_STEP_ATTR __attribute__((amdgpu_waves_per_eu(2)))
#include "meso_device.h"

namespace meso {

hipError_t launch_step_fast64(const Desc &d, int lim, int mode, int final_pass, int src,
                              hipStream_t st) {
    if (d.nc == 7) {
        if (lim == 1) launch_step_variants<double, double, 2, 1, 7>(d, mode, final_pass, src, st);
        else launch_step_variants<double, double, 2, 0, 7>(d, mode, final_pass, src, st);
    } else {
        if (lim == 1) launch_step_variants<double, double, 2, 1, 6>(d, mode, final_pass, src, st);
        else launch_step_variants<double, double, 2, 0, 6>(d, mode, final_pass, src, st);
    }
    return hipGetLastError();
}

hipError_t launch_batched_step_fast64(const Desc *descs, const int4 *tiles, int ntiles, int lim,
                                      int eos, int nc, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (nc == 7) launch_batched_variants<double, double, 2, 7>(descs, tiles, ntiles, lim, 1, st);
    else launch_batched_variants<double, double, 2, 6>(descs, tiles, ntiles, lim, eos, st);
    return hipGetLastError();
}

}  // namespace meso
