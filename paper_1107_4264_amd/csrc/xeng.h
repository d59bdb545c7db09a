// Internal interface between the host planner/ABI and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

namespace xc {

enum InFmt { IN_CI8 = 0, IN_CI4 = 1, IN_CF32 = 2 };
// ACC_F32M: fp32 matrix cores (v_mfma_f32_32x32x2_f32), the plain path's arithmetic on the
// matrix cores.  ACC_F6: fp6 e3m2 operands on the scaled f8f6f4 matrix cores.
enum AccPath { ACC_F32_CMAC = 0, ACC_I8 = 1, ACC_F16 = 2, ACC_F8 = 3, ACC_F32M = 4, ACC_F6 = 5 };
constexpr int ACC_LAST = ACC_F6;

// Largest |sample component| a low-precision operand type holds exactly: fp8 e4m3 every
// integer of [-16, 16], fp6 e3m2 every integer of [-8, 8]; 0 for the other paths (no limit
// below the sample format's).
constexpr int exact_operand_bound(int acc) { return acc == ACC_F8 ? 16 : (acc == ACC_F6 ? 8 : 0); }
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
    int staging;          // 0: operands staged in LDS; 1: loaded per wave through the caches
    int variant;          // compile-time variant of the whole-channel / super-tiled kernel
    int64_t nitems;       // nchan * tiles_per_chan * nwindows
    int64_t grid;         // blocks in this launch
    int64_t block0;       // item number of block 0 (launches are split below 2^24 blocks)
    void *work;           // fp6 super-tiles: the unit workspace (f6_work_bytes), else unused
};

// Bytes of the fp6 super-tiles' workspace: 48 bytes (the e3m2 codes of 32 samples) per
// (channel, block of 32 samples, input), the inputs padded to whole super-rows of 256.
inline size_t f6_work_bytes(int nin, int nchan, int ntime)
{
    const size_t npad = 256 * (size_t)((nin + 255) / 256), ntb = (size_t)((ntime + 31) / 32);
    return (size_t)nchan * ntb * npad * 48;
}

// One entry of a batch work list: job index, channel, tile, window.
struct XItem {
    int job;
    int chan;
    int tile;
    int window;
};

// Launchers (return a hipError_t as int).
int launch_mfma(const XJob &job, int acc, int in_fmt, hipStream_t stream);
// The tiled kernel without the LDS stage (operands loaded per wave through the caches).
int launch_mfma_cache(const XJob &job, int acc, int in_fmt, hipStream_t stream);
int launch_cmac(const XJob &job, int in_fmt, hipStream_t stream);
int launch_zero(void *ptr, size_t bytes, hipStream_t stream);
// Zero *count, then add the number of sample components of `in` (bytes of CI8, or of CI4
// when ci4) outside [-max_abs, max_abs] to it.
int launch_range_count(const void *in, size_t bytes, bool ci4, int max_abs, unsigned long long *count,
                       hipStream_t stream);
// Whole-channel kernel (tile 256): persistent, job.grid workgroups of 512 threads walk the
// job.nitems (channel, window) items, window-major.
int launch_chan(const XJob &job, int acc, hipStream_t stream);
// Super-tiles (tile 512): triangles, then rectangles, each at most `cus` workgroups; on the
// fp6 path (CI4) first the pre-pass into job.work (f6_work_bytes; required).
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

// Work list generated on the device instead of uploaded (for a job table in a fixed
// workspace): queue q holds, job after job in table order, the channels f of job j
// with (f + j) % NQUEUE == q, each as tiles_per_chan * nwindows items (window-major, the
// tiles of one (channel, window) adjacent).  qend[q * maxj + j] counts the items of queue q
// in jobs 0..j; qend[q * maxj + njobs - 1] is the queue's length.
struct XGenQueues {
    const int64_t *qend;
    int njobs;
    int maxj;
};

// Item `it` of queue q of a generated work list; false past the end of the queue.
__device__ __forceinline__ bool gen_item(const XJob *jobs, const XGenQueues &g, int q, int64_t it, XItem &item)
{
    const int64_t *e = g.qend + (int64_t)q * g.maxj;
    if (g.njobs <= 0 || it >= e[g.njobs - 1]) return false;
    int lo = 0, hi = g.njobs - 1;  // first job whose cumulative count exceeds it
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (e[mid] > it) hi = mid;
        else lo = mid + 1;
    }
    const XJob &jb = jobs[lo];
    const int64_t local = it - (lo > 0 ? e[lo - 1] : 0);
    const int64_t per_chan = (int64_t)jb.tiles_per_chan * jb.nwindows;
    const int64_t k = local / per_chan;
    const int64_t r = local - k * per_chan;
    const int f0 = ((q - lo) % NQUEUE + NQUEUE) % NQUEUE;
    item.job = lo;
    item.chan = (int)(f0 + (int64_t)NQUEUE * k);
    item.window = (int)(r / jb.tiles_per_chan);
    item.tile = (int)(r - (int64_t)item.window * jb.tiles_per_chan);
    return true;
}

int launch_mfma_batch(const XJob *jobs_dev, const XItem *items_dev, const XQueues &queues,
                      unsigned int *counters_dev, int acc, int in_fmt, int tile, int load_mode, int nblocks,
                      hipStream_t stream);
int launch_cmac_batch(const XJob *jobs_dev, const XItem *items_dev, const XQueues &queues,
                      unsigned int *counters_dev, int in_fmt, int nblocks, hipStream_t stream);
// The same persistent launches over a generated work list (counters zeroed by the caller).
int launch_mfma_batch_gen(const XJob *jobs_dev, const XGenQueues &g, unsigned int *counters_dev, int acc,
                          int in_fmt, int tile, int load_mode, int nblocks, hipStream_t stream);
int launch_cmac_batch_gen(const XJob *jobs_dev, const XGenQueues &g, unsigned int *counters_dev, int in_fmt,
                          int nblocks, hipStream_t stream);

// Fixed workspace of the batch entry point that allocates nothing (one per device, for the
// life of the process): queue counters, the generated work list's cumulative counts
// (NQUEUE x NOALLOC_MAX_JOBS int64) and the job table (NOALLOC_MAX_JOBS XJob).
constexpr int NOALLOC_MAX_JOBS = 256;
constexpr size_t NOALLOC_COUNTERS_OFF = 0;
constexpr size_t NOALLOC_QEND_OFF = 512;
constexpr size_t NOALLOC_JOBS_OFF = NOALLOC_QEND_OFF + (size_t)NQUEUE * NOALLOC_MAX_JOBS * sizeof(int64_t);
constexpr size_t NOALLOC_BYTES = NOALLOC_JOBS_OFF + (size_t)NOALLOC_MAX_JOBS * sizeof(XJob);
static_assert(NQUEUE * COUNTER_STRIDE * sizeof(unsigned int) <= NOALLOC_QEND_OFF, "counters fit");
static_assert(NOALLOC_JOBS_OFF % 16 == 0, "job table alignment");

// Device address of that workspace on the current device, looked up (hipGetSymbolAddress)
// the first time each device asks; a hipError_t as int.
int noalloc_scratch(void **ptr);

// Fill the workspace at `scratch` (a device address from noalloc_scratch) on `stream`: the
// job table (the XJobs travel as kernel arguments, a few per launch, so nothing is read
// from host memory after the call), then the generated queues' cumulative counts and zeroed
// counters.  ntab <= NOALLOC_MAX_JOBS.
int launch_noalloc_setup(void *scratch, const XJob *table, int ntab, hipStream_t stream);


// F-engine (fengine.hip): per input and frame an nchan-point DFT of the complex 8-bit
// samples in[nin][nsamp] (frame t = samples t nchan .. t nchan + nchan - 1), times gain,
// written corner-turned as out[t][k][i]: requantised int8 (re, im) pairs, or with `spectra`
// the complex fp32 values.  nchan a power of two in 64..2048.
int launch_fengine(const void *in, void *out, int nin, int nchan, int64_t nsamp, int nframes, float gain,
                   bool spectra, hipStream_t stream);

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
