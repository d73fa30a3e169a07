// meso_kernels_fp32.hip -- state-update kernels of the pure FP32 mode (inert
// liquids).  Built with floating-point contraction and the ILP-maximising
// instruction scheduler, which this mode's kernels take at no loss of
// occupancy (2 % faster); the FP32-bulk kernels (meso_kernels_fast.hip) would
// lose their third wave per SIMD to it.

#include "meso_device.h"

namespace meso {

hipError_t launch_step_fp32(const Desc &d, int lim, int mode, int final_pass, int src,
                            hipStream_t st) {
    if (lim == 1) launch_step_variants<float, float, true, 1, 6>(d, mode, final_pass, src, st);
    else launch_step_variants<float, float, true, 0, 6>(d, mode, final_pass, src, st);
    return hipGetLastError();
}

hipError_t launch_batched_step_fp32(const Desc *descs, const int4 *tiles, int ntiles, int lim,
                                    int eos, hipStream_t st) {
    launch_batched_variants<float, float, true, 6>(descs, tiles, ntiles, lim, eos, st);
    return hipGetLastError();
}

}  // namespace meso
