// meso_kernels_react_fast.hip -- step kernels of a reactive liquid in the
// FP32-bulk / FP64-accumulate and pure FP32 modes (built with floating-point
// contraction, like the inert kernels of these modes).

#include "meso_device.h"

namespace meso {

hipError_t launch_step_react_fast(const Desc &d, int prec, int lim, int mode, int final_pass,
                                  int src, hipStream_t st) {
    if (prec == kPMix) {
        if (lim == 1) launch_step_variants<double, float, true, 1, 7>(d, mode, final_pass, src, st);
        else launch_step_variants<double, float, true, 0, 7>(d, mode, final_pass, src, st);
    } else {
        if (lim == 1) launch_step_variants<float, float, true, 1, 7>(d, mode, final_pass, src, st);
        else launch_step_variants<float, float, true, 0, 7>(d, mode, final_pass, src, st);
    }
    return hipGetLastError();
}

hipError_t launch_batched_step_react_fast(const Desc *descs, const int4 *tiles, int ntiles,
                                          int prec, int lim, hipStream_t st) {
    if (prec == kPMix)
        launch_batched_variants<double, float, true, 7>(descs, tiles, ntiles, lim, 1, st);
    else
        launch_batched_variants<float, float, true, 7>(descs, tiles, ntiles, lim, 1, st);
    return hipGetLastError();
}

}  // namespace meso
