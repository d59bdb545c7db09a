// Internal interface between the host planner/ABI and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

namespace xc {

enum InFmt { IN_CI8 = 0, IN_CI4 = 1, IN_CF32 = 2 };
enum AccPath { ACC_F32_CMAC = 0, ACC_I8 = 1, ACC_F16 = 2, ACC_F8 = 3 };
enum OutFmt { OUT_CI32 = 0, OUT_CI64 = 1, OUT_C64 = 2, OUT_C128 = 3 };

// Global-load width the staging code may use for a job (fixed per job by nin alignment).
enum LoadMode { LOAD_VEC = 0, LOAD_WORD = 1, LOAD_ELEM = 2 };

// One correlation job as the kernels see it.  Items are (channel, tile, window) triples.
struct XJob {
    const void *in;       // [ntime][nchan][nin] samples
    void *out;            // [nchan][nbl][npol*npol] complex of the output type
    int nin;              // stations * polarisations
    int npol;
    int nchan;
    int ntime;
    int tile;             // inputs per tile side
    int ntile_side;       // ceil(nin / tile)
    int tiles_per_chan;   // ntile_side * (ntile_side + 1) / 2
    int window;           // samples per accumulation window
    int nwindows;         // ceil(ntime / window)
    int accumulate;       // 1: add each window into the (pre-zeroed) wide output
    int load_mode;        // LoadMode
    int xcd_group;        // 8: keep all tiles of a channel on one XCD; 1: plain order
    int64_t nitems;       // nchan * tiles_per_chan * nwindows
    int64_t grid;         // blocks in this launch
    int64_t block0;       // item number of block 0 (launches are split below 2^24 blocks)
};

// One entry of a batch work list: job index, channel, tile, window.
struct XItem {
    int job;
    int chan;
    int tile;
    int window;
};

// Launchers (return a hipError_t as int).
int launch_mfma(const XJob &job, int acc, int in_fmt, hipStream_t stream);
int launch_cmac(const XJob &job, int in_fmt, hipStream_t stream);
int launch_zero(void *ptr, size_t bytes, hipStream_t stream);
// Whole-channel kernel (tile 256): persistent, job.grid workgroups of 512 threads walk the
// job.nitems (channel, window) items, window-major.
int launch_chan(const XJob &job, int acc, hipStream_t stream);
int launch_super(const XJob &job, int acc, int in_fmt, int cus, hipStream_t stream);

// Batched persistent launch.  The work list is split into NQUEUE queues (one per XCD: a
// channel's items all go to one queue); workgroup b takes items from queue b % NQUEUE
// through an atomic counter, then steals from the other queues, and exits when all are
// empty.  counters_dev holds NQUEUE counters spaced COUNTER_STRIDE words apart, zeroed
// before every launch.
constexpr int NQUEUE = 8;
constexpr int COUNTER_STRIDE = 16;
struct XQueues {
    int64_t begin[NQUEUE];
    int64_t end[NQUEUE];
};

int launch_mfma_batch(const XJob *jobs_dev, const XItem *items_dev, const XQueues &queues,
                      unsigned int *counters_dev, int acc, int in_fmt, int tile, int load_mode, int nblocks,
                      hipStream_t stream);
int launch_cmac_batch(const XJob *jobs_dev, const XItem *items_dev, const XQueues &queues,
                      unsigned int *counters_dev, int in_fmt, int nblocks, hipStream_t stream);

// Number of compute units of the current device (for persistent grids).
int device_cus();

// Raise the dynamic-LDS limit of `Kernel` to `bytes` on the current device, once per device
// (the attribute belongs to the device that is current when it is set; one flag bit per
// device, devices past 63 set it at every launch).
template <auto Kernel>
int allow_lds_on_device(int bytes)
{
    static std::atomic<uint64_t> done{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    const uint64_t bit = dev >= 0 && dev < 64 ? (uint64_t)1 << dev : 0;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return 0;
    e = hipFuncSetAttribute((const void *)Kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return (int)e;
    done.fetch_or(bit, std::memory_order_acq_rel);
    return 0;
}

}  // namespace xc
