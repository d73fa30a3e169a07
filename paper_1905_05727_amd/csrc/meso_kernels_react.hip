// meso_kernels_react.hip -- step kernels of a reactive liquid (seven conserved
// components: the reactant mass z2 rho2 lambda is advected with the flow and
// reacts in the pointwise stage), FP64 mode.  Built without floating-point
// contraction, like the inert FP64 kernels.
//
// The seventh component's y-pipeline registers push the fused kernel to 276
// VGPRs, one wave per SIMD; it is compiled for two waves instead (256 VGPRs,
// 18 spilled to scratch), which hides more of the FP64 latency than the
// spills cost.

#define MESO_STEP_ATTR __attribute__((amdgpu_waves_per_eu(2)))
#include "meso_device.h"

namespace meso {

hipError_t launch_step_react(const Desc &d, int prec, int lim, int mode, int final_pass, int src,
                             hipStream_t st) {
    if (prec != kP64) return launch_step_react_fast(d, prec, lim, mode, final_pass, src, st);
    if (lim == 1) launch_step_variants<double, double, false, 1, 7>(d, mode, final_pass, src, st);
    else launch_step_variants<double, double, false, 0, 7>(d, mode, final_pass, src, st);
    return hipGetLastError();
}

hipError_t launch_batched_step_react(const Desc *descs, const int4 *tiles, int ntiles, int prec,
                                     int lim, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (prec != kP64) return launch_batched_step_react_fast(descs, tiles, ntiles, prec, lim, st);
    launch_batched_variants<double, double, false, 7>(descs, tiles, ntiles, lim, 1, st);
    return hipGetLastError();
}

}  // namespace meso
