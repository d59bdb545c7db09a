// X-engine on the CDNA4 matrix cores (gfx950).
//
// For one channel the visibilities are V = X X^H with X[i][t] = x_i(t) (Sec. 2.1, Eq. 4).
// Writing every complex sample as the real pair (re, im) along the contraction axis, the
// real part of V_ij is the real dot product of the pair sequences of inputs i and j, and
// the imaginary part is the dot product of input i's pairs with input j's pairs rotated to
// (-im, re).  Both are plain real matrix products with K = 2 * samples, so one tile of the
// triangle is two MFMA accumulations (real and imaginary) sharing the row operand: exactly
// four real MACs, i.e. the 8 flops of one complex MAC (Eq. 5), per input pair and sample.
//
// Tiling follows the multi-level idea of Sec. 2.2 / 4.1 with gfx950 levels:
//   * a workgroup owns one TILE x TILE square of the lower triangle (triangular tile
//     numbering of Sec. 4.2) for one channel and one accumulation window;
//   * its four waves own (TILE/2)^2 sub-squares; each wave holds 32x32 MFMA accumulator
//     blocks, the register level of the hierarchy;
//   * the row and column input vectors of a time block are staged in LDS (Sec. 4.4's
//     software-managed cache), double buffered so that one barrier per block suffices;
//   * on diagonal tiles, waves and 32x32 blocks strictly above the diagonal are skipped
//     (the wasted diagonal work of Sec. 6.1 is cut to the 32x32 granularity).
//
// LDS holds, per time group of G samples and input, one 16-byte unit (two for fp8):
// the G samples' (re, im) pairs in the operand type, which is exactly what one lane of an
// MFMA needs; rows are XOR-swizzled by time group so that stores and loads are free of
// bank conflicts.

#include <hip/hip_runtime.h>

#include "xeng.h"

namespace xc {
namespace {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

constexpr int NTHREADS = 256;

template <int ACC>
struct Op;
// G: samples per lane per MFMA (one lane-half of K); WORDS: 32-bit words per lane operand;
// TB: samples per staged time block.
template <>
struct Op<ACC_I8> {
    static constexpr int G = 8, WORDS = 4, TB = 64;
    using acc_t = i32x16;
};
template <>
struct Op<ACC_F16> {
    static constexpr int G = 4, WORDS = 4, TB = 32;
    using acc_t = f32x16;
};
template <>
struct Op<ACC_F8> {
    static constexpr int G = 16, WORDS = 8, TB = 64;
    using acc_t = f32x16;
};

template <int W>
struct Frag {
    uint32_t w[W];
};

__device__ __forceinline__ void mma(i32x16 &c, const Frag<4> &a, const Frag<4> &b)
{
    i32x4 av = {(int)a.w[0], (int)a.w[1], (int)a.w[2], (int)a.w[3]};
    i32x4 bv = {(int)b.w[0], (int)b.w[1], (int)b.w[2], (int)b.w[3]};
    c = __builtin_amdgcn_mfma_i32_32x32x32_i8(av, bv, c, 0, 0, 0);
}

__device__ __forceinline__ void mma(f32x16 &c, const Frag<4> &a, const Frag<4> &b)
{
    i32x4 av = {(int)a.w[0], (int)a.w[1], (int)a.w[2], (int)a.w[3]};
    i32x4 bv = {(int)b.w[0], (int)b.w[1], (int)b.w[2], (int)b.w[3]};
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, av),
                                               __builtin_bit_cast(f16x8, bv), c, 0, 0, 0);
}

__device__ __forceinline__ void mma(f32x16 &c, const Frag<8> &a, const Frag<8> &b)
{
    i32x8 av, bv;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        av[k] = (int)a.w[k];
        bv[k] = (int)b.w[k];
    }
    // Formats 0/0 = fp8 e4m3 for both operands; E8M0 scale 127 = 2^0 for both.
    c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, 127, 0, 127);
}

// (re, im) pairs of a column operand -> (-im, re): the column of the imaginary product.
template <int ACC>
__device__ __forceinline__ uint32_t rotate_pairs(uint32_t w);

template <>
__device__ __forceinline__ uint32_t rotate_pairs<ACC_I8>(uint32_t w)
{
    const uint32_t s = __builtin_amdgcn_perm(w, w, 0x02030001u);  // [im0 re0 im1 re1]
    const i16x2 n = (i16x2){0, 0} - __builtin_bit_cast(i16x2, s);  // low bytes negated
    return (__builtin_bit_cast(uint32_t, n) & 0x00FF00FFu) | (s & 0xFF00FF00u);
}

template <>
__device__ __forceinline__ uint32_t rotate_pairs<ACC_F16>(uint32_t w)
{
    return __builtin_amdgcn_perm(w, w, 0x01000302u) ^ 0x00008000u;
}

template <>
__device__ __forceinline__ uint32_t rotate_pairs<ACC_F8>(uint32_t w)
{
    return __builtin_amdgcn_perm(w, w, 0x02030001u) ^ 0x00800080u;
}

__device__ __forceinline__ int sext4(uint32_t v) { return ((int)(v << 28)) >> 28; }

// ---------------------------------------------------------------- sample decoding

template <int IN>
struct InFmtT;
template <>
struct InFmtT<IN_CI8> {
    static constexpr int BPC = 2;  // bytes per complex sample
};
template <>
struct InFmtT<IN_CI4> {
    static constexpr int BPC = 1;
};

// Signed (re, im) of input e of a loaded row (words w).
template <int IN, int LW>
__device__ __forceinline__ void pair_of(const uint32_t (&w)[LW], int e, int &re, int &im)
{
    if constexpr (IN == IN_CI8) {
        const uint32_t h = w[e >> 1] >> ((e & 1) * 16);
        re = (int)(int8_t)(h & 0xFF);
        im = (int)(int8_t)((h >> 8) & 0xFF);
    } else {
        const uint32_t b = w[e >> 2] >> ((e & 3) * 8);
        re = sext4((b >> 4) & 0xF);
        im = sext4(b & 0xF);
    }
}

__device__ __forceinline__ uint32_t f16_bits(int v)
{
    return (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)(short)v);
}

// ---------------------------------------------------------------- the tile kernel body

template <int ACC, int IN, int TILE>
struct Tile {
    using O = Op<ACC>;
    using acc_t = typename O::acc_t;
    static constexpr int G = O::G;
    static constexpr int TB = O::TB;
    static constexpr int WORDS = O::WORDS;
    static constexpr int PLANES = WORDS / 4;
    static constexpr int NTG = TB / G;                       // time groups per block
    static constexpr int SWZ = (NTG < 8 ? NTG : 8) - 1;      // row swizzle mask
    static constexpr int BPC = InFmtT<IN>::BPC;
    static constexpr int CI = (ACC == ACC_F8 && IN == IN_CI8) ? 4 : 8;  // inputs per load
    static constexpr int LW = CI * BPC / 4;                  // words per row load
    static constexpr int NT = NTG * (TILE / CI);             // staging tasks per side
    static constexpr int NB = TILE / 64;                     // 32x32 blocks per wave side
    static constexpr int WT = TILE / 2;                      // wave sub-tile side
    static constexpr int SIDE_BYTES = NTG * PLANES * TILE * 16;
    static constexpr int LDS_BYTES = 2 * 2 * SIDE_BYTES;     // 2 buffers x 2 sides
    static_assert(NT <= 128 || TILE > 128, "one staging task per thread and side");
    static_assert(TB % (2 * G) == 0, "time block holds whole K-steps");
};

template <int ACC, int IN, int TILE>
__device__ __forceinline__ void load_task(const XJob &p, int f, int side_row0, int t0, int t_end,
                                          int tg, int chunk,
                                          uint32_t (&rows)[Tile<ACC, IN, TILE>::G][Tile<ACC, IN, TILE>::LW])
{
    using T = Tile<ACC, IN, TILE>;
    const uint8_t *in = (const uint8_t *)p.in;
    const int i0 = side_row0 + chunk * T::CI;
#pragma unroll
    for (int u = 0; u < T::G; ++u) {
        const int t = t0 + tg * T::G + u;
#pragma unroll
        for (int k = 0; k < T::LW; ++k) rows[u][k] = 0u;
        if (t >= t_end || i0 >= p.nin) continue;
        const uint8_t *src = in + (((int64_t)t * p.nchan + f) * p.nin + i0) * T::BPC;
        if (p.load_mode == LOAD_VEC) {
            if constexpr (T::LW == 4) {
                const uint4 v = *(const uint4 *)src;
                rows[u][0] = v.x; rows[u][1] = v.y; rows[u][2] = v.z; rows[u][3] = v.w;
            } else {
                const uint2 v = *(const uint2 *)src;
                rows[u][0] = v.x; rows[u][1] = v.y;
            }
        } else if (p.load_mode == LOAD_WORD) {
            constexpr int PER_WORD = 4 / T::BPC;
#pragma unroll
            for (int k = 0; k < T::LW; ++k)
                if (i0 + k * PER_WORD < p.nin) rows[u][k] = *(const uint32_t *)(src + 4 * k);
        } else {
#pragma unroll
            for (int b = 0; b < T::LW * 4; ++b)
                if (i0 + b / T::BPC < p.nin) rows[u][b >> 2] |= (uint32_t)src[b] << (8 * (b & 3));
        }
    }
}

// Pack input e of a task's loaded rows into its LDS unit (WORDS words).
template <int ACC, int IN, int TILE>
__device__ __forceinline__ void pack_unit(
    const uint32_t (&rows)[Tile<ACC, IN, TILE>::G][Tile<ACC, IN, TILE>::LW], int e,
    uint32_t (&u)[Tile<ACC, IN, TILE>::WORDS])
{
    using T = Tile<ACC, IN, TILE>;
    if constexpr (ACC == ACC_I8) {
        if constexpr (IN == IN_CI8) {
            const uint32_t sel = (e & 1) ? 0x07060302u : 0x05040100u;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                u[m] = __builtin_amdgcn_perm(rows[2 * m + 1][e >> 1], rows[2 * m][e >> 1], sel);
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                int r0, i0, r1, i1;
                pair_of<IN>(rows[2 * m], e, r0, i0);
                pair_of<IN>(rows[2 * m + 1], e, r1, i1);
                u[m] = (uint32_t)(r0 & 0xFF) | ((uint32_t)(i0 & 0xFF) << 8) |
                       ((uint32_t)(r1 & 0xFF) << 16) | ((uint32_t)(i1 & 0xFF) << 24);
            }
        }
    } else if constexpr (ACC == ACC_F16) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int re, im;
            pair_of<IN>(rows[m], e, re, im);
            u[m] = f16_bits(re) | (f16_bits(im) << 16);
        }
    } else {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int r0, i0, r1, i1;
            pair_of<IN>(rows[2 * m], e, r0, i0);
            pair_of<IN>(rows[2 * m + 1], e, r1, i1);
            uint32_t w = __builtin_amdgcn_cvt_pk_fp8_f32((float)r0, (float)i0, 0, false);
            u[m] = __builtin_amdgcn_cvt_pk_fp8_f32((float)r1, (float)i1, w, true);
        }
    }
}

template <int ACC, int IN, int TILE>
__device__ __forceinline__ uint32_t lds_off(int side, int tg, int plane, int row)
{
    using T = Tile<ACC, IN, TILE>;
    return (uint32_t)(side * T::SIDE_BYTES +
                      ((tg * T::PLANES + plane) * TILE + (row ^ (tg & T::SWZ))) * 16);
}

template <int ACC, int IN, int TILE>
__device__ __forceinline__ void process_item(const XJob &p, int f, int g, int w, uint8_t *lds)
{
    using T = Tile<ACC, IN, TILE>;
    using acc_t = typename T::acc_t;
    constexpr int NB = T::NB;

    // Triangular tile index -> (bx, by), bx <= by (Sec. 4.2), exact integer fix-up.
    int by = (int)((sqrtf(8.0f * (float)g + 1.0f) - 1.0f) * 0.5f);
    while (by * (by + 1) / 2 > g) --by;
    while ((by + 1) * (by + 2) / 2 <= g) ++by;
    const int bx = g - by * (by + 1) / 2;
    const bool diag = (bx == by);
    const int row0 = by * TILE, col0 = bx * TILE;
    const int t_begin = w * p.window;
    const int t_end = min(p.ntime, t_begin + p.window);
    const int nblk = (t_end - t_begin + T::TB - 1) / T::TB;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    // Which 32x32 blocks of this wave are computed.
    bool on[NB][NB];
    bool any = false;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int rbi = wr * NB + a, cbi = wc * NB + b;
            on[a][b] = !(diag && rbi < cbi) && (row0 + rbi * 32 < p.nin) && (col0 + cbi * 32 < p.nin);
            any |= on[a][b];
        }

    acc_t re[NB][NB], im[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            re[a][b] = (acc_t){};
            im[a][b] = (acc_t){};
        }

    // Staging task of this thread: side, time group, input chunk.
    const int nsides = diag ? 1 : 2;
    const bool has_task = tid < nsides * T::NT;
    const int side = tid / T::NT;
    const int task = tid - side * T::NT;
    const int tg = task % T::NTG;
    const int chunk = task / T::NTG;
    const int side_row0 = side == 0 ? row0 : col0;
    uint32_t rows[T::G][T::LW];

    auto stage_store = [&](int buf) {
        if (!has_task) return;
        uint8_t *base = lds + buf * 2 * T::SIDE_BYTES;
#pragma unroll
        for (int e = 0; e < T::CI; ++e) {
            uint32_t u[T::WORDS];
            pack_unit<ACC, IN, TILE>(rows, e, u);
#pragma unroll
            for (int pl = 0; pl < T::PLANES; ++pl) {
                uint4 v = {u[4 * pl], u[4 * pl + 1], u[4 * pl + 2], u[4 * pl + 3]};
                *(uint4 *)(base + lds_off<ACC, IN, TILE>(side, tg, pl, chunk * T::CI + e)) = v;
            }
        }
    };

    if (has_task) load_task<ACC, IN, TILE>(p, f, side_row0, t_begin, t_end, tg, chunk, rows);
    stage_store(0);
    __syncthreads();

    const int col_side = diag ? 0 : 1;
    const int r32 = lane & 31, half = lane >> 5;

    for (int blk = 0; blk < nblk; ++blk) {
        const int cur = blk & 1;
        const bool next = blk + 1 < nblk;
        if (next && has_task)
            load_task<ACC, IN, TILE>(p, f, side_row0, t_begin + (blk + 1) * T::TB, t_end, tg,
                                     chunk, rows);
        if (any) {
            const uint8_t *base = lds + cur * 2 * T::SIDE_BYTES;
#pragma unroll
            for (int s = 0; s < T::NTG / 2; ++s) {
                const int tgk = 2 * s + half;
                Frag<T::WORDS> A[NB], B[NB], C[NB];
#pragma unroll
                for (int a = 0; a < NB; ++a) {
                    const int row = (wr * NB + a) * 32 + r32;
#pragma unroll
                    for (int pl = 0; pl < T::PLANES; ++pl) {
                        const uint4 v = *(const uint4 *)(base + lds_off<ACC, IN, TILE>(0, tgk, pl, row));
                        A[a].w[4 * pl] = v.x; A[a].w[4 * pl + 1] = v.y;
                        A[a].w[4 * pl + 2] = v.z; A[a].w[4 * pl + 3] = v.w;
                    }
                }
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int col = (wc * NB + b) * 32 + r32;
#pragma unroll
                    for (int pl = 0; pl < T::PLANES; ++pl) {
                        const uint4 v = *(const uint4 *)(base + lds_off<ACC, IN, TILE>(col_side, tgk, pl, col));
                        B[b].w[4 * pl] = v.x; B[b].w[4 * pl + 1] = v.y;
                        B[b].w[4 * pl + 2] = v.z; B[b].w[4 * pl + 3] = v.w;
                    }
#pragma unroll
                    for (int k = 0; k < T::WORDS; ++k) C[b].w[k] = rotate_pairs<ACC>(B[b].w[k]);
                }
#pragma unroll
                for (int a = 0; a < NB; ++a)
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        if (on[a][b]) {
                            mma(re[a][b], A[a], B[b]);
                            mma(im[a][b], A[a], C[b]);
                        }
            }
        }
        if (next) stage_store(cur ^ 1);
        __syncthreads();
    }

    // Epilogue: lane holds column r32 of each block, rows 8*(k/4) + 4*half + k%4.
    const int npol = p.npol;
    const int64_t nbl = (int64_t)(p.nin / npol) * (p.nin / npol + 1) / 2;
    const int npp = npol * npol;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (!on[a][b]) continue;
            const int j = col0 + (wc * NB + b) * 32 + r32;
            if (j >= p.nin) continue;
            const int s2 = j / npol, q = j - s2 * npol;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int i = row0 + (wr * NB + a) * 32 + 8 * (k >> 2) + 4 * half + (k & 3);
                if (i >= p.nin) continue;
                const int s1 = i / npol, pp = i - s1 * npol;
                if (s1 < s2) continue;
                const int64_t o = (((int64_t)f * nbl + (int64_t)s1 * (s1 + 1) / 2 + s2) * npp +
                                   pp * npol + q) * 2;
                if constexpr (ACC == ACC_I8) {
                    if (p.accumulate) {
                        long long *out = (long long *)p.out;
                        atomicAdd((unsigned long long *)&out[o], (unsigned long long)(long long)re[a][b][k]);
                        atomicAdd((unsigned long long *)&out[o + 1], (unsigned long long)(long long)im[a][b][k]);
                    } else {
                        int2 v = {re[a][b][k], im[a][b][k]};
                        *(int2 *)((int *)p.out + o) = v;
                    }
                } else {
                    if (p.accumulate) {
                        double *out = (double *)p.out;
                        atomicAdd(&out[o], (double)re[a][b][k]);
                        atomicAdd(&out[o + 1], (double)im[a][b][k]);
                    } else {
                        float2 v = {re[a][b][k], im[a][b][k]};
                        *(float2 *)((float *)p.out + o) = v;
                    }
                }
            }
        }
}

// Item b of a single job -> (channel, tile, window).  With xcd_group 8, the workgroups of
// channel f all get b % 8 == f % 8, i.e. the same XCD under round-robin dispatch, so the
// tiles that re-read a channel's inputs share one L2.
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

template <int ACC, int IN, int TILE>
__global__ __launch_bounds__(NTHREADS, 2) void xeng_mfma_kernel(XJob p)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[Tile<ACC, IN, TILE>::LDS_BYTES];
    int f, g, w;
    if (!decode_item(p, p.block0 + blockIdx.x, f, g, w)) return;
    process_item<ACC, IN, TILE>(p, f, g, w, lds);
}

// Persistent batched kernel: workgroups take (job, channel, tile, window) items off a
// global counter until the list is exhausted; every workgroup reaches the exit.
template <int ACC, int IN, int TILE>
__global__ __launch_bounds__(NTHREADS, 2) void xeng_mfma_batch_kernel(const XJob *jobs, const XItem *items,
                                                                      int64_t nitems, unsigned int *counter)
{
    __shared__ __attribute__((aligned(16))) uint8_t lds[Tile<ACC, IN, TILE>::LDS_BYTES];
    __shared__ int64_t next;
    for (;;) {
        if (threadIdx.x == 0) next = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t it = next;
        __syncthreads();
        if (it >= nitems) break;
        const XItem item = items[it];
        const XJob p = jobs[item.job];
        process_item<ACC, IN, TILE>(p, item.chan, item.tile, item.window, lds);
    }
}

template <int ACC, int IN, int TILE>
int launch_one(const XJob &job, hipStream_t stream)
{
    hipLaunchKernelGGL((xeng_mfma_kernel<ACC, IN, TILE>), dim3((unsigned)job.grid), dim3(NTHREADS), 0,
                       stream, job);
    return (int)hipGetLastError();
}

template <int ACC, int IN, int TILE>
int launch_batch(const XJob *jobs, const XItem *items, int64_t nitems, unsigned int *counter,
                 int nblocks, hipStream_t stream)
{
    hipLaunchKernelGGL((xeng_mfma_batch_kernel<ACC, IN, TILE>), dim3(nblocks), dim3(NTHREADS), 0,
                       stream, jobs, items, nitems, counter);
    return (int)hipGetLastError();
}

template <int ACC, int IN>
int launch_tile(const XJob &job, hipStream_t stream)
{
    if (job.tile == 128) return launch_one<ACC, IN, 128>(job, stream);
    if (job.tile == 64) return launch_one<ACC, IN, 64>(job, stream);
    return (int)hipErrorInvalidValue;
}

template <int ACC>
int launch_in(const XJob &job, int in_fmt, hipStream_t stream)
{
    if (in_fmt == IN_CI8) return launch_tile<ACC, IN_CI8>(job, stream);
    if (in_fmt == IN_CI4) return launch_tile<ACC, IN_CI4>(job, stream);
    return (int)hipErrorInvalidValue;
}

template <int ACC, int IN>
int launch_batch_tile(const XJob *jobs, const XItem *items, int64_t n, unsigned int *counter,
                      int tile, int nblocks, hipStream_t stream)
{
    if (tile == 128) return launch_batch<ACC, IN, 128>(jobs, items, n, counter, nblocks, stream);
    if (tile == 64) return launch_batch<ACC, IN, 64>(jobs, items, n, counter, nblocks, stream);
    return (int)hipErrorInvalidValue;
}

template <int ACC>
int launch_batch_in(const XJob *jobs, const XItem *items, int64_t n, unsigned int *counter, int in_fmt,
                    int tile, int nblocks, hipStream_t stream)
{
    if (in_fmt == IN_CI8) return launch_batch_tile<ACC, IN_CI8>(jobs, items, n, counter, tile, nblocks, stream);
    if (in_fmt == IN_CI4) return launch_batch_tile<ACC, IN_CI4>(jobs, items, n, counter, tile, nblocks, stream);
    return (int)hipErrorInvalidValue;
}

}  // namespace

int launch_mfma(const XJob &job, int acc, int in_fmt, hipStream_t stream)
{
    if (job.grid <= 0) return 0;
    switch (acc) {
    case ACC_I8: return launch_in<ACC_I8>(job, in_fmt, stream);
    case ACC_F16: return launch_in<ACC_F16>(job, in_fmt, stream);
    case ACC_F8: return launch_in<ACC_F8>(job, in_fmt, stream);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_mfma_batch(const XJob *jobs_dev, const XItem *items_dev, int64_t nitems,
                      unsigned int *counter_dev, int acc, int in_fmt, int tile, int nblocks,
                      hipStream_t stream)
{
    if (nitems <= 0) return 0;
    switch (acc) {
    case ACC_I8: return launch_batch_in<ACC_I8>(jobs_dev, items_dev, nitems, counter_dev, in_fmt, tile, nblocks, stream);
    case ACC_F16: return launch_batch_in<ACC_F16>(jobs_dev, items_dev, nitems, counter_dev, in_fmt, tile, nblocks, stream);
    case ACC_F8: return launch_batch_in<ACC_F8>(jobs_dev, items_dev, nitems, counter_dev, in_fmt, tile, nblocks, stream);
    default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace xc
