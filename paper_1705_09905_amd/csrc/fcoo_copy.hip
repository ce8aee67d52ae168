// A plain device-to-device copy: the bandwidth ceiling the sparse kernels are
// measured against on the same GPU, and the kernel of known traffic that
// hardware byte counters (FETCH_SIZE, WRITE_SIZE) are calibrated on.
#include <hip/hip_runtime.h>

#include "fcoo_internal.h"

namespace fcoo {
namespace dev {

// One pass: workgroup b copies the contiguous 16 KB block b (256 threads x 4
// elements of 16 bytes, streaming loads and stores), so the grid holds one
// workgroup per block.  On an MI355X this shape moved 1 GiB at 6.3 TB/s
// (read + write) where a grid-stride loop over a capped grid reached 4.3-5.2
// and hipMemcpyAsync 4.9.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kCopyPer = 4;                            // elements per thread

__global__ __launch_bounds__(256) void copy_kernel(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst, int64_t n)
{
    const int64_t b = (int64_t)blockIdx.x * (256 * kCopyPer) + threadIdx.x;
    u32x4 v[kCopyPer];
#pragma unroll
    for (int u = 0; u < kCopyPer; ++u)
        if (b + u * 256 < n) v[u] = __builtin_nontemporal_load(src + b + u * 256);
#pragma unroll
    for (int u = 0; u < kCopyPer; ++u)
        if (b + u * 256 < n) __builtin_nontemporal_store(v[u], dst + b + u * 256);
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
    const int64_t g = (n + 256 * dev::kCopyPer - 1) / (256 * dev::kCopyPer);
    if (g > 0x7fffffff) return fail(FCOO_EINVAL, "bytes = %lld: too large for one launch", (long long)bytes);
    hipLaunchKernelGGL(dev::copy_kernel, dim3((unsigned)g), dim3(256), 0, (hipStream_t)stream,
                       static_cast<const dev::u32x4 *>(src), static_cast<dev::u32x4 *>(dst), n);
    FCOO_HIP(hipGetLastError());
    return FCOO_OK;
}
