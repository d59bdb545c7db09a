// Dispatch of the tiled matrix-core X-engine launches to the translation unit of each
// arithmetic path (xeng_mfma_<path>.hip; kernels in xeng_mfma_impl.h).
#include <hip/hip_runtime.h>

#include "xeng.h"

namespace xc {

int launch_mfma_i8(const XJob &job, int in_fmt, hipStream_t stream);
int launch_mfma_cache_i8(const XJob &job, int in_fmt, hipStream_t stream);
int launch_mfma_batch_i8(const XJob *jobs, const XItem *items, const XQueues &q, unsigned int *counters, int in_fmt,
                          int tile, int mode, int nblocks, hipStream_t stream);
int launch_mfma_batch_gen_i8(const XJob *jobs, const XGenQueues &g, unsigned int *counters, int in_fmt, int tile,
                              int mode, int nblocks, hipStream_t stream);
int launch_mfma_f16(const XJob &job, int in_fmt, hipStream_t stream);
int launch_mfma_cache_f16(const XJob &job, int in_fmt, hipStream_t stream);
int launch_mfma_batch_f16(const XJob *jobs, const XItem *items, const XQueues &q, unsigned int *counters, int in_fmt,
                          int tile, int mode, int nblocks, hipStream_t stream);
int launch_mfma_batch_gen_f16(const XJob *jobs, const XGenQueues &g, unsigned int *counters, int in_fmt, int tile,
                              int mode, int nblocks, hipStream_t stream);
int launch_mfma_f8(const XJob &job, int in_fmt, hipStream_t stream);
int launch_mfma_cache_f8(const XJob &job, int in_fmt, hipStream_t stream);
int launch_mfma_batch_f8(const XJob *jobs, const XItem *items, const XQueues &q, unsigned int *counters, int in_fmt,
                          int tile, int mode, int nblocks, hipStream_t stream);
int launch_mfma_batch_gen_f8(const XJob *jobs, const XGenQueues &g, unsigned int *counters, int in_fmt, int tile,
                              int mode, int nblocks, hipStream_t stream);
int launch_mfma_f32m(const XJob &job, int in_fmt, hipStream_t stream);
int launch_mfma_cache_f32m(const XJob &job, int in_fmt, hipStream_t stream);
int launch_mfma_batch_f32m(const XJob *jobs, const XItem *items, const XQueues &q, unsigned int *counters, int in_fmt,
                          int tile, int mode, int nblocks, hipStream_t stream);
int launch_mfma_batch_gen_f32m(const XJob *jobs, const XGenQueues &g, unsigned int *counters, int in_fmt, int tile,
                              int mode, int nblocks, hipStream_t stream);
int launch_mfma_f6(const XJob &job, int in_fmt, hipStream_t stream);
int launch_mfma_cache_f6(const XJob &job, int in_fmt, hipStream_t stream);
int launch_mfma_batch_f6(const XJob *jobs, const XItem *items, const XQueues &q, unsigned int *counters, int in_fmt,
                          int tile, int mode, int nblocks, hipStream_t stream);
int launch_mfma_batch_gen_f6(const XJob *jobs, const XGenQueues &g, unsigned int *counters, int in_fmt, int tile,
                              int mode, int nblocks, hipStream_t stream);

int launch_mfma(const XJob &job, int acc, int in_fmt, hipStream_t stream)
{
    if (job.grid <= 0) return 0;
    switch (acc) {
    case ACC_I8: return launch_mfma_i8(job, in_fmt, stream);
    case ACC_F16: return launch_mfma_f16(job, in_fmt, stream);
    case ACC_F8: return launch_mfma_f8(job, in_fmt, stream);
    case ACC_F32M: return launch_mfma_f32m(job, in_fmt, stream);
    case ACC_F6: return launch_mfma_f6(job, in_fmt, stream);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_mfma_cache(const XJob &job, int acc, int in_fmt, hipStream_t stream)
{
    if (job.grid <= 0) return 0;
    switch (acc) {
    case ACC_I8: return launch_mfma_cache_i8(job, in_fmt, stream);
    case ACC_F16: return launch_mfma_cache_f16(job, in_fmt, stream);
    case ACC_F8: return launch_mfma_cache_f8(job, in_fmt, stream);
    case ACC_F32M: return launch_mfma_cache_f32m(job, in_fmt, stream);
    case ACC_F6: return launch_mfma_cache_f6(job, in_fmt, stream);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_mfma_batch(const XJob *jobs_dev, const XItem *items_dev, const XQueues &queues,
                      unsigned int *counters_dev, int acc, int in_fmt, int tile, int load_mode, int nblocks,
                      hipStream_t stream)
{
    if (nblocks <= 0) return 0;
    switch (acc) {
    case ACC_I8: return launch_mfma_batch_i8(jobs_dev, items_dev, queues, counters_dev, in_fmt, tile, load_mode, nblocks, stream);
    case ACC_F16: return launch_mfma_batch_f16(jobs_dev, items_dev, queues, counters_dev, in_fmt, tile, load_mode, nblocks, stream);
    case ACC_F8: return launch_mfma_batch_f8(jobs_dev, items_dev, queues, counters_dev, in_fmt, tile, load_mode, nblocks, stream);
    case ACC_F32M: return launch_mfma_batch_f32m(jobs_dev, items_dev, queues, counters_dev, in_fmt, tile, load_mode, nblocks, stream);
    case ACC_F6: return launch_mfma_batch_f6(jobs_dev, items_dev, queues, counters_dev, in_fmt, tile, load_mode, nblocks, stream);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_mfma_batch_gen(const XJob *jobs_dev, const XGenQueues &g, unsigned int *counters_dev, int acc,
                          int in_fmt, int tile, int load_mode, int nblocks, hipStream_t stream)
{
    if (nblocks <= 0) return 0;
    switch (acc) {
    case ACC_I8: return launch_mfma_batch_gen_i8(jobs_dev, g, counters_dev, in_fmt, tile, load_mode, nblocks, stream);
    case ACC_F16: return launch_mfma_batch_gen_f16(jobs_dev, g, counters_dev, in_fmt, tile, load_mode, nblocks, stream);
    case ACC_F8: return launch_mfma_batch_gen_f8(jobs_dev, g, counters_dev, in_fmt, tile, load_mode, nblocks, stream);
    case ACC_F32M: return launch_mfma_batch_gen_f32m(jobs_dev, g, counters_dev, in_fmt, tile, load_mode, nblocks, stream);
    case ACC_F6: return launch_mfma_batch_gen_f6(jobs_dev, g, counters_dev, in_fmt, tile, load_mode, nblocks, stream);
    default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace xc
