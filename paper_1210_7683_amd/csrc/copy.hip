// Device -> pinned host copy kernel for the b sink: 16-byte loads from device
// memory and 16-byte stores into host memory mapped into the device's address
// space, over a fixed number of workgroups (so the copy shares the chip with
// concurrent launches instead of waiting for free hardware engines). Each
// thread fences its stores to system scope before the kernel ends, so the
// host may read the data once the kernel's completion event has fired.
#include "gwas_internal.h"

namespace gw {
namespace {

__global__ __launch_bounds__(256) void copy_to_host_kernel(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                           int64_t n16, uint32_t *__restrict__ dst_tail,
                                                           const uint32_t *__restrict__ src_tail, int tail) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n16; k += stride) dst[k] = src[k];
    if (blockIdx.x == 0 && threadIdx.x < tail) dst_tail[threadIdx.x] = src_tail[threadIdx.x];
    __threadfence_system();
}

}  // namespace

hipError_t launch_copy_to_host(void *dst_dev_view, const void *src, int64_t bytes, int grid, hipStream_t s) {
    if (bytes <= 0) return hipSuccess;
    if ((bytes & 3) || (((uintptr_t)dst_dev_view | (uintptr_t)src) & 15)) return hipErrorInvalidValue;
    const int64_t n16 = bytes / 16;
    const int tail = (int)((bytes - n16 * 16) / 4);
    hipLaunchKernelGGL(copy_to_host_kernel, dim3(grid), dim3(256), 0, s, (uint4 *)dst_dev_view, (const uint4 *)src,
                       n16, (uint32_t *)((uint8_t *)dst_dev_view + n16 * 16),
                       (const uint32_t *)((const uint8_t *)src + n16 * 16), tail);
    return hipGetLastError();
}

}  // namespace gw
