// Fixed device workspace of the batch entry point that allocates nothing
// (xcorr_batch_run_noalloc): a file-scope device array, one copy per GPU, held until the
// process ends.  Host code never passes the array's name to a kernel or a copy (in host code
// it names a host-side stand-in, not device memory): it looks up the device address once
// per device with that device current and uses that address everywhere.

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>

#include "xeng.h"

namespace xc {
namespace {

static __device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

// Jobs per table-writing launch (their kernel arguments stay well below the 4 KiB limit).
constexpr int JOBS_PER_LAUNCH = 10;
struct TableChunk {
    int first;
    int n;
    XJob jobs[JOBS_PER_LAUNCH];
};

__global__ __launch_bounds__(64) void table_kernel(uint8_t *ws, TableChunk c)
{
    XJob *t = (XJob *)(ws + NOALLOC_JOBS_OFF);
    if ((int)threadIdx.x < c.n) t[c.first + threadIdx.x] = c.jobs[threadIdx.x];
}

// One thread per queue: cumulative item counts of the generated work list (see XGenQueues:
// channel f of table job j is in queue (f + j) % NQUEUE), and the queue counters zeroed.
__global__ __launch_bounds__(64) void queues_kernel(uint8_t *ws, int ntab)
{
    const int q = threadIdx.x;
    if (q >= NQUEUE) return;
    const XJob *t = (const XJob *)(ws + NOALLOC_JOBS_OFF);
    int64_t *e = (int64_t *)(ws + NOALLOC_QEND_OFF) + (int64_t)q * NOALLOC_MAX_JOBS;
    int64_t sum = 0;
    for (int j = 0; j < ntab; ++j) {
        const int f0 = ((q - j) % NQUEUE + NQUEUE) % NQUEUE;
        const int64_t chans = t[j].nchan > f0 ? (t[j].nchan - f0 + NQUEUE - 1) / NQUEUE : 0;
        sum += chans * t[j].tiles_per_chan * t[j].nwindows;
        e[j] = sum;
    }
    ((unsigned int *)(ws + NOALLOC_COUNTERS_OFF))[q * COUNTER_STRIDE] = 0u;
}

constexpr int MAX_DEVICES = 64;
std::atomic<void *> g_scratch_ptr[MAX_DEVICES];
std::mutex g_scratch_mu;

}  // namespace

int noalloc_scratch(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
    void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return (int)e;
            if (!p) return (int)hipErrorInvalidSymbol;
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *ptr = p;
    return 0;
}

int launch_noalloc_setup(void *scratch, const XJob *table, int ntab, hipStream_t stream)
{
    if (ntab < 0 || ntab > NOALLOC_MAX_JOBS) return (int)hipErrorInvalidValue;
    uint8_t *ws = (uint8_t *)scratch;
    for (int first = 0; first < ntab; first += JOBS_PER_LAUNCH) {
        TableChunk c;
        c.first = first;
        c.n = ntab - first < JOBS_PER_LAUNCH ? ntab - first : JOBS_PER_LAUNCH;
        for (int k = 0; k < c.n; ++k) c.jobs[k] = table[first + k];
        hipLaunchKernelGGL(table_kernel, dim3(1), dim3(64), 0, stream, ws, c);
        if (hipError_t e = hipGetLastError(); e != hipSuccess) return (int)e;
    }
    hipLaunchKernelGGL(queues_kernel, dim3(1), dim3(64), 0, stream, ws, ntab);
    return (int)hipGetLastError();
}

}  // namespace xc
