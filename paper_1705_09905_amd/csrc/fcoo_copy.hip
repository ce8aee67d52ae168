// A plain device-to-device copy: the bandwidth ceiling the sparse kernels are
// measured against on the same GPU, and the kernel of known traffic that
// hardware byte counters (FETCH_SIZE, WRITE_SIZE) are calibrated on.
#include <hip/hip_runtime.h>

#include "fcoo_internal.h"

namespace fcoo {
namespace dev {

// 16-byte elements, four loads in flight per thread, grid-stride.
__global__ __launch_bounds__(256) void copy_kernel(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace dev
}  // namespace fcoo

using namespace fcoo;

extern "C" int fcoo_device_copy(const void *src, void *dst, int64_t bytes, void *stream)
{
    clear_error();
    if (bytes < 0 || bytes % 16) return fail(FCOO_EINVAL, "bytes = %lld must be a non-negative multiple of 16",
                                             (long long)bytes);
    if (bytes == 0) return FCOO_OK;
    if (!src || !dst) return fail(FCOO_EINVAL, "src or dst is NULL");
    if (((uintptr_t)src | (uintptr_t)dst) & 15) return fail(FCOO_EINVAL, "src and dst must be 16-byte aligned");
    const int64_t n = bytes / 16;
    int64_t g = (n + 256 * 4 - 1) / (256 * 4);
    if (g > 256 * 16) g = 256 * 16;                   // 16 workgroups per CU, then grid-stride
    hipLaunchKernelGGL(dev::copy_kernel, dim3((unsigned)g), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
    FCOO_HIP(hipGetLastError());
    return FCOO_OK;
}
