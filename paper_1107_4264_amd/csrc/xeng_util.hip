// Small device utilities: a fill kernel that zeroes the wide output before windows are
// summed into it (a kernel rather than hipMemsetAsync, so that the work can be captured in
// a HIP graph and replayed), and the optional range check of integer samples.

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

// Components outside [-m, m]: a CI8 byte is one two's-complement component, a CI4 byte
// holds the real part in its high nibble and the imaginary part in its low nibble.
template <bool CI4>
__device__ __forceinline__ unsigned out_of_range(uint32_t w, int m)
{
    unsigned n = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t byte = (w >> (8 * b)) & 0xFFu;
        if constexpr (CI4) {
            const int hi = (int)(byte >> 4) - (int)((byte >> 3) & 0x10u);
            const int lo = (int)(byte & 0xFu) - (int)((byte << 1) & 0x10u);
            n += (hi > m || hi < -m) + (lo > m || lo < -m);
        } else {
            const int v = (int)(int8_t)byte;
            n += (v > m || v < -m);
        }
    }
    return n;
}

// One pass over the input: 16-byte words of the aligned body (grid-stride), the bytes
// before and after it by the first block.  Threads with a count add it to *count.
template <bool CI4>
__global__ __launch_bounds__(256) void range_kernel(const uint4 *body, size_t n16, const uint8_t *head, int nhead,
                                                    const uint8_t *tail, int ntail, int m,
                                                    unsigned long long *count)
{
    unsigned n = 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride) {
        const uint4 v = body[k];
        n += out_of_range<CI4>(v.x, m) + out_of_range<CI4>(v.y, m) + out_of_range<CI4>(v.z, m) +
             out_of_range<CI4>(v.w, m);
    }
    if (blockIdx.x == 0) {
        if ((int)threadIdx.x < nhead) n += out_of_range<CI4>(head[threadIdx.x], m);
        if ((int)threadIdx.x < ntail) n += out_of_range<CI4>(tail[threadIdx.x], m);
    }
    if (n) atomicAdd(count, (unsigned long long)n);
}

}  // namespace

int launch_range_count(const void *in, size_t bytes, bool ci4, int max_abs, unsigned long long *count,
                       hipStream_t stream)
{
    if (int rc = launch_zero(count, sizeof(unsigned long long), stream)) return rc;
    if (bytes == 0) return 0;
    const uintptr_t a = (uintptr_t)in;
    const size_t head = ((16 - (a & 15)) & 15) < bytes ? ((16 - (a & 15)) & 15) : bytes;
    const uint8_t *body = (const uint8_t *)in + head;
    const size_t n16 = (bytes - head) / 16;
    const size_t ntail = bytes - head - n16 * 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks == 0) blocks = 1;
    if (ci4)
        hipLaunchKernelGGL(range_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, stream, (const uint4 *)body, n16,
                           (const uint8_t *)in, (int)head, body + n16 * 16, (int)ntail, max_abs, count);
    else
        hipLaunchKernelGGL(range_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, stream, (const uint4 *)body, n16,
                           (const uint8_t *)in, (int)head, body + n16 * 16, (int)ntail, max_abs, count);
    return (int)hipGetLastError();
}

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
