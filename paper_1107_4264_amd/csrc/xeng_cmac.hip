// The paper's X-engine arithmetic: FP32 complex multiply-accumulate on the vector ALUs.
//
// Structure as in Sec. 4.2 and 4.4 (the software-managed cache kernel), re-sized for
// gfx950: the lower triangle is cut into 64x64 input tiles numbered in triangular order
// (Sec. 4.2); a workgroup of 256 threads (4 waves) owns one tile of one channel and one
// accumulation window; each thread holds a 4x4 register tile of complex accumulators
// (R = 4 in the paper's notation, T = 16x16 threads, RT = 64); the row and column input
// vectors of each block of time samples are converted to float and staged in LDS, double
// buffered so that one barrier per block suffices (the "Buf" variant of Table 3).  Like the
// paper's kernel, threads of a diagonal tile compute their whole register tile and only
// pairs on or below the diagonal are stored (Sec. 4.4).
//
// Per complex MAC: re += ar*br + ai*bi, im += ai*br - ar*bi (4 FMAs, the 8 flops of Eq. 5).
//
// Float samples are summed in two levels: each staged block of TB samples goes into fresh
// partial sums that are then added to the running sums.  A recursive fp32 sum of n terms
// errs by up to about n u of the magnitude sum (u = 2^-24); two levels cut n from 2T to
// 2 TB + T / TB.  Integer samples need no such care: below 2^24 every fp32 partial sum of
// integers is exact (the accumulation windows keep them there).

#include <hip/hip_runtime.h>

#include "xeng.h"

namespace xc {
namespace {

constexpr int NTHREADS = 256;
constexpr int TILE = 64;
constexpr int TB = 16;   // samples per staged block
constexpr int RT = 4;    // register tile side

template <int IN>
__device__ __forceinline__ void load_samples(const XJob &p, int f, int t, int i0, float2 (&v)[4])
{
    // Four consecutive inputs i0..i0+3 of channel f at time t, as floats (zero outside).
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = make_float2(0.f, 0.f);
    if (t < 0 || i0 >= p.nin) return;
    const int64_t n = ((int64_t)t * p.nchan + f) * p.nin + i0;
    if constexpr (IN == IN_CF32) {
        const float2 *src = (const float2 *)p.in + n;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k < p.nin) v[k] = src[k];
    } else if constexpr (IN == IN_CI8) {
        const int8_t *src = (const int8_t *)p.in + 2 * n;
        if (p.load_mode == LOAD_VEC) {
            const uint2 w = *(const uint2 *)src;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t h = (k < 2 ? w.x : w.y) >> ((k & 1) * 16);
                v[k] = make_float2((float)(int8_t)(h & 0xFF), (float)(int8_t)(h >> 8));
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (i0 + k < p.nin) v[k] = make_float2((float)src[2 * k], (float)src[2 * k + 1]);
        }
    } else {
        const uint8_t *src = (const uint8_t *)p.in + n;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k < p.nin) {
                const uint32_t b = src[k];
                v[k] = make_float2((float)(((int)(b << 24)) >> 28), (float)(((int)(b << 28)) >> 28));
            }
    }
}

template <int IN>
__device__ __forceinline__ void process_item(const XJob &p, int f, int g, int w, float2 *lds)
{
    int by = (int)((sqrtf(8.0f * (float)g + 1.0f) - 1.0f) * 0.5f);
    while (by * (by + 1) / 2 > g) --by;
    while ((by + 1) * (by + 2) / 2 <= g) ++by;
    const int bx = g - by * (by + 1) / 2;
    const bool diag = (bx == by);
    const int row0 = by * TILE, col0 = bx * TILE;
    const int t_begin = w * p.window;
    const int t_end = min(p.ntime, t_begin + p.window);
    const int nblk = (t_end - t_begin + TB - 1) / TB;

    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;

    float accr[RT][RT], acci[RT][RT];
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < RT; ++b) accr[a][b] = acci[a][b] = 0.f;

    // Staging: thread loads 4 inputs of one sample per side; 256 threads x 4 = TB x TILE.
    const int st = tid >> 4;          // sample within block
    const int sc = (tid & 15) * 4;    // first input within tile
    float2 vr[4], vc[4];
    constexpr int SIDE = TB * TILE;   // float2 per side per buffer

    auto load = [&](int t0) {
        const int t = t0 + st;
        const int tt = t < t_end ? t : -1;
        load_samples<IN>(p, f, tt, row0 + sc, vr);
        if (!diag) load_samples<IN>(p, f, tt, col0 + sc, vc);
    };
    auto store = [&](int buf) {
        float4 *dst = (float4 *)(lds + buf * 2 * SIDE + st * TILE + sc);
        dst[0] = make_float4(vr[0].x, vr[0].y, vr[1].x, vr[1].y);
        dst[1] = make_float4(vr[2].x, vr[2].y, vr[3].x, vr[3].y);
        if (!diag) {
            float4 *dc = (float4 *)(lds + buf * 2 * SIDE + SIDE + st * TILE + sc);
            dc[0] = make_float4(vc[0].x, vc[0].y, vc[1].x, vc[1].y);
            dc[1] = make_float4(vc[2].x, vc[2].y, vc[3].x, vc[3].y);
        }
    };

    load(t_begin);
    store(0);
    __syncthreads();
    const int cside = diag ? 0 : SIDE;
    for (int blk = 0; blk < nblk; ++blk) {
        const int cur = blk & 1;
        const bool next = blk + 1 < nblk;
        if (next) load(t_begin + (blk + 1) * TB);
        const float2 *rb = lds + cur * 2 * SIDE;
        const float2 *cb = rb + cside;
        auto mac_block = [&](float (&sr)[RT][RT], float (&si)[RT][RT]) __attribute__((always_inline)) {
#pragma unroll 4
            for (int s = 0; s < TB; ++s) {
                float2 x[RT], y[RT];
#pragma unroll
                for (int a = 0; a < RT; ++a) x[a] = rb[s * TILE + ty + 16 * a];
#pragma unroll
                for (int b = 0; b < RT; ++b) y[b] = cb[s * TILE + tx + 16 * b];
#pragma unroll
                for (int a = 0; a < RT; ++a)
#pragma unroll
                    for (int b = 0; b < RT; ++b) {
                        sr[a][b] = fmaf(x[a].x, y[b].x, sr[a][b]);
                        sr[a][b] = fmaf(x[a].y, y[b].y, sr[a][b]);
                        si[a][b] = fmaf(x[a].y, y[b].x, si[a][b]);
                        si[a][b] = fmaf(-x[a].x, y[b].y, si[a][b]);
                    }
            }
        };
        if constexpr (IN == IN_CF32) {
            float pr[RT][RT], pi[RT][RT];
#pragma unroll
            for (int a = 0; a < RT; ++a)
#pragma unroll
                for (int b = 0; b < RT; ++b) pr[a][b] = pi[a][b] = 0.f;
            mac_block(pr, pi);
#pragma unroll
            for (int a = 0; a < RT; ++a)
#pragma unroll
                for (int b = 0; b < RT; ++b) {
                    accr[a][b] += pr[a][b];
                    acci[a][b] += pi[a][b];
                }
        } else {
            mac_block(accr, acci);
        }
        if (next) store(cur ^ 1);
        __syncthreads();
    }

    const int npol = p.npol;
    const int64_t nbl = (int64_t)(p.nin / npol) * (p.nin / npol + 1) / 2;
    const int npp = npol * npol;
#pragma unroll
    for (int a = 0; a < RT; ++a) {
        const int i = row0 + ty + 16 * a;
        if (i >= p.nin) continue;
        const int s1 = i / npol, pp = i - s1 * npol;
#pragma unroll
        for (int b = 0; b < RT; ++b) {
            const int j = col0 + tx + 16 * b;
            if (j >= p.nin) continue;
            const int s2 = j / npol, q = j - s2 * npol;
            if (s1 < s2) continue;
            const int64_t o = (((int64_t)f * nbl + (int64_t)s1 * (s1 + 1) / 2 + s2) * npp + pp * npol + q) * 2;
            if (p.accumulate) {
                double *out = (double *)p.out;
                atomicAdd(&out[o], (double)accr[a][b]);
                atomicAdd(&out[o + 1], (double)acci[a][b]);
            } else {
                *(float2 *)((float *)p.out + o) = make_float2(accr[a][b], acci[a][b]);
            }
        }
    }
}

__device__ __forceinline__ bool decode_item(const XJob &p, int64_t b, int &f, int &g, int &w)
{
    const int64_t per_chan = (int64_t)p.tiles_per_chan * p.nwindows;
    int64_t r;
    if (p.xcd_group == 8) {
        const int64_t q = b >> 3;
        const int64_t grp = q / per_chan;
        r = q - grp * per_chan;
        f = (int)(grp * 8 + (b & 7));
    } else {
        f = (int)(b / per_chan);
        r = b - (int64_t)f * per_chan;
    }
    if (f >= p.nchan) return false;
    w = (int)(r / p.tiles_per_chan);
    g = (int)(r - (int64_t)w * p.tiles_per_chan);
    return true;
}

template <int IN>
__global__ __launch_bounds__(NTHREADS) void xeng_cmac_kernel(XJob p)
{
    __shared__ __attribute__((aligned(16))) float2 lds[2 * 2 * TB * TILE];
    int f, g, w;
    if (!decode_item(p, p.block0 + blockIdx.x, f, g, w)) return;
    process_item<IN>(p, f, g, w, lds);
}

template <int IN>
__global__ __launch_bounds__(NTHREADS) void xeng_cmac_batch_kernel(const XJob *jobs, const XItem *items, XQueues q,
                                                                   unsigned int *counters)
{
    __shared__ __attribute__((aligned(16))) float2 lds[2 * 2 * TB * TILE];
    __shared__ int64_t next;
    const int q0 = blockIdx.x % NQUEUE;
    for (int qi = 0; qi < NQUEUE; ++qi) {
        const int qq = (q0 + qi) % NQUEUE;
        for (;;) {
            if (threadIdx.x == 0) next = q.begin[qq] + (int64_t)atomicAdd(&counters[qq * COUNTER_STRIDE], 1u);
            __syncthreads();
            const int64_t it = next;
            __syncthreads();
            if (it >= q.end[qq]) break;
            const XItem item = items[it];
            const XJob jb = jobs[item.job];  // a register copy (see the tiled batch kernel)
            process_item<IN>(jb, item.chan, item.tile, item.window, lds);
        }
    }
}

template <int IN>
__global__ __launch_bounds__(NTHREADS) void xeng_cmac_batch_gen_kernel(const XJob *jobs, XGenQueues gq,
                                                                       unsigned int *counters)
{
    __shared__ __attribute__((aligned(16))) float2 lds[2 * 2 * TB * TILE];
    __shared__ int64_t next;
    const int q0 = blockIdx.x % NQUEUE;
    for (int qi = 0; qi < NQUEUE; ++qi) {
        const int qq = (q0 + qi) % NQUEUE;
        for (;;) {
            if (threadIdx.x == 0) next = (int64_t)atomicAdd(&counters[qq * COUNTER_STRIDE], 1u);
            __syncthreads();
            const int64_t it = next;
            __syncthreads();
            XItem item;
            if (!gen_item(jobs, gq, qq, it, item)) break;
            const XJob jb = jobs[item.job];  // a register copy (see the tiled batch kernel)
            process_item<IN>(jb, item.chan, item.tile, item.window, lds);
        }
    }
}

}  // namespace

int launch_cmac(const XJob &job, int in_fmt, hipStream_t stream)
{
    if (job.grid <= 0) return 0;
    const dim3 grid((unsigned)job.grid), block(NTHREADS);
    switch (in_fmt) {
    case IN_CI8: hipLaunchKernelGGL(xeng_cmac_kernel<IN_CI8>, grid, block, 0, stream, job); break;
    case IN_CI4: hipLaunchKernelGGL(xeng_cmac_kernel<IN_CI4>, grid, block, 0, stream, job); break;
    case IN_CF32: hipLaunchKernelGGL(xeng_cmac_kernel<IN_CF32>, grid, block, 0, stream, job); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_cmac_batch(const XJob *jobs_dev, const XItem *items_dev, const XQueues &queues,
                      unsigned int *counters_dev, int in_fmt, int nblocks, hipStream_t stream)
{
    if (nblocks <= 0) return 0;
    const dim3 grid(nblocks), block(NTHREADS);
    switch (in_fmt) {
    case IN_CI8: hipLaunchKernelGGL(xeng_cmac_batch_kernel<IN_CI8>, grid, block, 0, stream, jobs_dev, items_dev, queues, counters_dev); break;
    case IN_CI4: hipLaunchKernelGGL(xeng_cmac_batch_kernel<IN_CI4>, grid, block, 0, stream, jobs_dev, items_dev, queues, counters_dev); break;
    case IN_CF32: hipLaunchKernelGGL(xeng_cmac_batch_kernel<IN_CF32>, grid, block, 0, stream, jobs_dev, items_dev, queues, counters_dev); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int launch_cmac_batch_gen(const XJob *jobs_dev, const XGenQueues &g, unsigned int *counters_dev, int in_fmt,
                          int nblocks, hipStream_t stream)
{
    if (nblocks <= 0) return 0;
    const dim3 grid(nblocks), block(NTHREADS);
    switch (in_fmt) {
    case IN_CI8: hipLaunchKernelGGL(xeng_cmac_batch_gen_kernel<IN_CI8>, grid, block, 0, stream, jobs_dev, g, counters_dev); break;
    case IN_CI4: hipLaunchKernelGGL(xeng_cmac_batch_gen_kernel<IN_CI4>, grid, block, 0, stream, jobs_dev, g, counters_dev); break;
    case IN_CF32: hipLaunchKernelGGL(xeng_cmac_batch_gen_kernel<IN_CF32>, grid, block, 0, stream, jobs_dev, g, counters_dev); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

}  // namespace xc
