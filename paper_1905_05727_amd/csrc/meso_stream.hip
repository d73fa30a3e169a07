// meso_stream.hip -- a plain device-to-device copy, the reference a
// measurement holds the state-update kernels against: one read and one write
// per byte, as in the algorithmic traffic of a step, at the highest rate this
// kernel reaches on the device.

#include "meso.h"
#include "meso_internal.h"

namespace meso {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// Each thread moves U 16-byte vectors per trip (all loads issued before the
// first store), grid-stride over the whole vectors; a ragged tail of fewer
// than 16 bytes is copied byte by byte by the first workgroup.
template <int U, bool NT>
__global__ __launch_bounds__(256) void stream_copy_kernel(const v4u *__restrict__ src,
                                                          v4u *__restrict__ dst, size_t nvec,
                                                          const unsigned char *__restrict__ tsrc,
                                                          unsigned char *__restrict__ tdst,
                                                          int ntail) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (U - 1) * stride < nvec; i += U * stride) {
        v4u v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = NT ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (NT) __builtin_nontemporal_store(v[u], dst + i + u * stride);
            else dst[i + u * stride] = v[u];
        }
    }
    for (; i < nvec; i += stride) dst[i] = src[i];
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tdst[threadIdx.x] = tsrc[threadIdx.x];
}

}  // namespace meso

extern "C" int32_t mf_stream_copy(const void *src, void *dst, size_t bytes, int32_t variant,
                                  int32_t workgroups, void *hip_stream) {
    if ((!src || !dst) && bytes) return MF_E_INVALID_ARG;
    if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return MF_E_INVALID_ARG;
    if (variant < 0 || variant > 3 || workgroups < 0) return MF_E_INVALID_ARG;
    if (bytes == 0) return MF_OK;
    const size_t nvec = bytes / 16;
    const int ntail = (int)(bytes % 16);
    int wg = workgroups;
    if (wg == 0) {
        const int cus = meso::device_cus();
        wg = 8 * (cus > 0 ? cus : 256);
    }
    const size_t need = (nvec + 255) / 256;
    if ((size_t)wg > need) wg = need > 0 ? (int)need : 1;
    const meso::v4u *s = (const meso::v4u *)src;
    meso::v4u *d = (meso::v4u *)dst;
    const unsigned char *ts = (const unsigned char *)src + nvec * 16;
    unsigned char *td = (unsigned char *)dst + nvec * 16;
    hipStream_t st = (hipStream_t)hip_stream;
    void (*k)(const meso::v4u *, meso::v4u *, size_t, const unsigned char *, unsigned char *, int);
    switch (variant) {
        case 0: k = meso::stream_copy_kernel<1, false>; break;
        case 1: k = meso::stream_copy_kernel<4, false>; break;
        case 2: k = meso::stream_copy_kernel<1, true>; break;
        default: k = meso::stream_copy_kernel<4, true>; break;
    }
    hipLaunchKernelGGL(k, dim3(wg), dim3(256), 0, st, s, d, nvec, ts, td, ntail);
    return hipGetLastError() == hipSuccess ? MF_OK : MF_E_DEVICE;
}
