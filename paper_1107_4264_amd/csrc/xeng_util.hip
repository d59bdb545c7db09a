// Small device utilities: a fill kernel that zeroes the wide output before windows are
// summed into it.  A kernel rather than hipMemsetAsync, so that the work can be captured in
// a HIP graph and replayed.

#include <hip/hip_runtime.h>

#include "xeng.h"

namespace xc {
namespace {

__global__ __launch_bounds__(256) void zero_kernel(uint4 *p16, size_t n16, uint8_t *tail, size_t ntail)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride)
        p16[k] = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

}  // namespace

int launch_zero(void *ptr, size_t bytes, hipStream_t stream)
{
    if (bytes == 0) return 0;
    // Output buffers come from the caller; only 16-byte multiples go through the wide path.
    const uintptr_t a = (uintptr_t)ptr;
    const size_t head = (16 - (a & 15)) & 15;
    if (head) {
        // Misaligned start: clear byte-wise in one block.
        hipLaunchKernelGGL(zero_kernel, dim3(1), dim3(256), 0, stream, (uint4 *)nullptr, (size_t)0,
                           (uint8_t *)ptr, head < bytes ? head : bytes);
        if (head >= bytes) return (int)hipGetLastError();
    }
    uint8_t *body = (uint8_t *)ptr + head;
    const size_t rest = bytes - head;
    const size_t n16 = rest / 16;
    const size_t ntail = rest - n16 * 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, (uint4 *)body, n16,
                       body + n16 * 16, ntail);
    return (int)hipGetLastError();
}

int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

}  // namespace xc
