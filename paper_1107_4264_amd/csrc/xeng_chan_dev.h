// Device pieces shared by the whole-channel kernel (xeng_chan.hip) and the super-tiled
// kernel (xeng_super.hip): the LDS copy ring, transposing operand reads, operand forms for
// the int8 / fp16 / fp8 matrix cores, the 32x32-block work lists, the pipelined K-step and
// the stores of a channel's triangle.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "xeng.h"
#include "xeng_dev.h"

#pragma clang diagnostic ignored "-Winline-asm"

namespace xc {
namespace {

using namespace dev;

constexpr int CT = 512;                         // eight waves, two per SIMD
constexpr int CROW = 512;                       // LDS bytes per time row (256 inputs)
constexpr uint32_t COOB = 0xFFFFFFF0u;          // offset beyond every descriptor

// Per path: TB time rows per block, RING raw blocks in the LDS ring, STAGE: the operands are
// converted once per block into an LDS buffer (two buffers) instead of at every fragment
// read.  The int8 path multiplies the raw pairs directly; the fp16 path converts each
// sample once (its conversion costs more than the transposing read it replaces).
template <int ACC>
struct ChanCfg;
template <>
struct ChanCfg<ACC_I8> {
    static constexpr int TB = 64, RING = 4;
    static constexpr bool STAGE = false;
};
template <>
struct ChanCfg<ACC_F16> {
    static constexpr int TB = 32, RING = 5;  // measured: 6 slots (the whole LDS) are slower
    static constexpr bool STAGE = true;
};
// Variant V (chosen by the autotuner): bit 0 keeps one block fewer in the LDS ring.
template <int ACC, int V = 0>
struct Geom {
    static constexpr int TB = ChanCfg<ACC>::TB, RING = ChanCfg<ACC>::RING - (V & 1);
    static constexpr bool STAGE = ChanCfg<ACC>::STAGE;
    static constexpr int BLK = TB * CROW;                   // raw bytes per block
    static constexpr int DPW = TB / 2 / (CT / 64);          // copies per wave per block
    static constexpr int QUADS = TB / 4;                    // 4-sample groups per block
    static constexpr int FBUF = STAGE ? QUADS * 256 * 16 : 0;  // staged operand bytes
    static constexpr int LDS = RING * BLK + 2 * FBUF;
    static_assert(LDS <= 160 * 1024, "LDS of one compute unit");
};

template <int ACC>
struct COp;
// KS: samples per K-step; NREAD: transposing reads per fragment (4 samples each); FW:
// 32-bit words of an MFMA operand fragment per lane.
template <>
struct COp<ACC_I8> {
    static constexpr int KS = 16, NREAD = 2, FW = 4;
    using acc_t = i32x16;
};
template <>
struct COp<ACC_F16> {
    static constexpr int KS = 8, NREAD = 1, FW = 4;
    using acc_t = f32x16;
};
// fp8 e4m3 (super-tiles only): 32x32x64 MFMAs, 32 samples per K-step
template <>
struct COp<ACC_F8> {
    static constexpr int KS = 32, NREAD = 4, FW = 8;
    using acc_t = f32x16;
};

typedef int i32x4s __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) s16x4 lds_s16x4;

// One row pair of a block: lane l copies 16 bytes at `voff` of the descriptor to LDS byte
// lds + 16 l.  Issued as inline assembly so that the compiler does not drain the whole
// ring (vmcnt 0) before every LDS read; completion is awaited explicitly (wait_dma).
__device__ __forceinline__ void dma16(i32x4s rsrc, uint32_t lds, uint32_t voff)
{
    asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds" ::"s"(lds), "v"(voff), "s"(rsrc)
                 : "memory", "m0");
}

// s_waitcnt vmcnt(N) (other counters untouched), N <= 63.
template <int N>
__device__ __forceinline__ void wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// ---------------------------------------------------------------- operands

template <int ACC>
struct Raw {
    uint32_t w[2 * COp<ACC>::NREAD];
};

// fp16 operand words of a raw fragment: (re, im) pairs, exactly.
__device__ __forceinline__ void f16_pairs(uint32_t w, uint32_t &p0, uint32_t &p1)
{
    ci8x2_to_f16(w, p0, p1);
}

template <int ACC>
__device__ __forceinline__ Frag<COp<ACC>::FW> op_plain(const Raw<ACC> &r)
{
    Frag<COp<ACC>::FW> o;
    if constexpr (ACC == ACC_I8 || ACC == ACC_F8) {
#pragma unroll
        for (int k = 0; k < COp<ACC>::FW; ++k) o.w[k] = r.w[k];
    } else {
        f16_pairs(r.w[0], o.w[0], o.w[1]);
        f16_pairs(r.w[1], o.w[2], o.w[3]);
    }
    return o;
}

// Rotated operands for the imaginary part, Im V_ij = sum_t (im_i re_j - re_i im_j): either
// the column operand as (-im, re) pairs (COL) or the row operand as (im, -re) pairs, from the
// plain operand words (int8, fp16 or fp8 e4m3 pairs), exactly.
template <int ACC, bool COL>
__device__ __forceinline__ Frag<COp<ACC>::FW> op_rot(const Frag<COp<ACC>::FW> &a)
{
    Frag<COp<ACC>::FW> o;
#pragma unroll
    for (int k = 0; k < COp<ACC>::FW; ++k) {
        if constexpr (ACC == ACC_F8) {
            // swap the bytes of each pair, then flip the sign bit of the component negated
            const uint32_t sw = __builtin_amdgcn_perm(a.w[k], a.w[k], 0x02030001u);
            o.w[k] = sw ^ (COL ? 0x00800080u : 0x80008000u);
        } else if constexpr (ACC == ACC_I8) {
            if constexpr (COL) {
                o.w[k] = rotate_pairs<ACC_I8>(a.w[k]);
            } else {
                // [im, re] per pair, then the high byte negated: (~re + 1) with the carry
                // leaving the 16-bit lane
                const uint32_t sw = __builtin_amdgcn_perm(a.w[k], a.w[k], 0x02030001u);
                const i16x2 v = __builtin_bit_cast(i16x2, sw ^ 0xFF00FF00u) + (i16x2){0x0100, 0x0100};
                o.w[k] = __builtin_bit_cast(uint32_t, v);
            }
        } else {
            // one packed multiply: low half = high half x sign.lo, high half = low half x
            // sign.hi (op_sel picks the swapped halves of the operand)
            const uint32_t sgn = COL ? 0x3C00BC00u : 0xBC003C00u;  // (-1, 1) or (1, -1)
            asm("v_pk_mul_f16 %0, %1, %2 op_sel:[1,0] op_sel_hi:[0,1]" : "=v"(o.w[k]) : "v"(a.w[k]), "s"(sgn));
        }
    }
    return o;
}

// Transposing reads of the fragment of block row R for K-step KSTEP from the ring slot
// whose per-lane addresses are lv[] (see lane_bases).
template <int ACC, int R, int KSTEP, int ROWB = CROW>
__device__ __forceinline__ Raw<ACC> read_frag(const uint32_t (&lv)[4])
{
    using O = COp<ACC>;
    Raw<ACC> r;
#pragma unroll
    for (int e = 0; e < O::NREAD; ++e) {
        const uint32_t imm = (uint32_t)((KSTEP * O::KS + 4 * e) * ROWB + 256 * (R >> 2));
        const s16x4 v = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_s16x4 *)(uintptr_t)(lv[R & 3] + imm));
        const uint2 u = __builtin_bit_cast(uint2, v);
        r.w[2 * e] = u.x;
        r.w[2 * e + 1] = u.y;
    }
    return r;
}

// Per-lane byte offsets (within a ring slot) of the transposing reads.  Lane l = 16g + 4k + a
// points at time row 4k' + k of its half (h = l / 32 selects samples 4*NREAD*h ..), input
// 32R + 16(g % 2) + 4a; chunk c = 4R + 2(g % 2) + a / 2 of the row sits at chunk c ^ 4k,
// i.e. at 4(R ^ k) + j: for R & 3 = q that is 64(q ^ k) + 16j, plus 256 for R >= 4.
template <int ACC, int ROWB = CROW>
__device__ __forceinline__ uint32_t lane_base(int lane, int q)
{
    using O = COp<ACC>;
    const int h = lane >> 5;
    const int k = (lane >> 2) & 3;
    const int j = 2 * ((lane >> 4) & 1) + ((lane & 3) >> 1);
    return (uint32_t)(h * 4 * O::NREAD * ROWB + k * ROWB + 64 * (q ^ k) + 16 * j + 8 * (lane & 1));
}

// ---------------------------------------------------------------- epilogue

// Store one 32x32 block with top-left input (row0, col0): lanes hold column col0 + lane % 32,
// register k holds row row0 + 8(k / 4) + 4(lane / 32) + k % 4.  Entries with an input
// beyond nin or with station s1 < s2 (the upper part of a diagonal block) are skipped.
// accumulate: add into the wide output with atomics (sums of windows).
template <int ACC>
__device__ __forceinline__ void store_block(void *out_ptr, int nin, int npol, int accumulate, int f, int row0,
                                            int col0, int lane, const typename COp<ACC>::acc_t &re,
                                            const typename COp<ACC>::acc_t &im)
{
    using val_t = typename std::conditional<ACC == ACC_I8, int, float>::type;
    using vec4_t = typename std::conditional<ACC == ACC_I8, i32x4v, f32x4>::type;
    if (row0 >= nin || col0 >= nin) return;
    const int r32 = lane & 31, half = lane >> 5;
    const int64_t nbl = (int64_t)(nin / npol) * (nin / npol + 1) / 2;
    const int j = col0 + r32;
    if (npol == 2 && !accumulate) {
        // lanes 2k, 2k+1 hold pols q = 0, 1 of one station; registers k, k+1 rows p = 0, 1:
        // after one exchange each lane stores the 16 bytes of one p row
        const bool odd = lane & 1;
        const int om = odd_lane_mask(lane);
        const int s2 = j >> 1;
#pragma unroll
        for (int k = 0; k < 16; k += 2) {
            const int i = row0 + 8 * (k >> 2) + 4 * half + (k & 3);
            const int s1 = i >> 1;
            const val_t r0 = (val_t)re[k], r1 = (val_t)re[k + 1];
            const val_t m0 = (val_t)im[k], m1 = (val_t)im[k + 1];
            const val_t xr = swap_pair_lanes(pair_send(r0, r1, om));
            const val_t xm = swap_pair_lanes(pair_send(m0, m1, om));
            if (i >= nin || j >= nin || s1 < s2) continue;
            const int64_t o = ((int64_t)f * nbl + (int64_t)s1 * (s1 + 1) / 2 + s2) * 8 + (odd ? 4 : 0);
            const vec4_t v = odd ? (vec4_t){xr, xm, r1, m1} : (vec4_t){r0, m0, xr, xm};
            __builtin_nontemporal_store(v, (vec4_t *)((val_t *)out_ptr + o));
        }
        return;
    }
    if (j >= nin) return;
    const int npp = npol * npol;
    const int s2 = j / npol, q = j - s2 * npol;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int i = row0 + 8 * (k >> 2) + 4 * half + (k & 3);
        if (i >= nin) continue;
        const int s1 = i / npol, pp = i - s1 * npol;
        if (s1 < s2) continue;
        const int64_t o = (((int64_t)f * nbl + (int64_t)s1 * (s1 + 1) / 2 + s2) * npp + pp * npol + q) * 2;
        if constexpr (ACC == ACC_I8) {
            if (accumulate) {
                unsigned long long *out = (unsigned long long *)out_ptr;
                atomicAdd(&out[o], (unsigned long long)(long long)re[k]);
                atomicAdd(&out[o + 1], (unsigned long long)(long long)im[k]);
            } else {
                *(int2 *)((int *)out_ptr + o) = make_int2(re[k], im[k]);
            }
        } else {
            if (accumulate) {
                double *out = (double *)out_ptr;
                atomicAdd(&out[o], (double)re[k]);
                atomicAdd(&out[o + 1], (double)im[k]);
            } else {
                *(float2 *)((float *)out_ptr + o) = make_float2(re[k], im[k]);
            }
        }
    }
}

// a <- (a lanes 0..31, b lanes 0..31), b <- (a lanes 32..63, b lanes 32..63).
__device__ __forceinline__ void lane_swap32(uint32_t &a, uint32_t &b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
}

__device__ __forceinline__ uint32_t bits32(int x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t bits32(float x) { return __builtin_bit_cast(uint32_t, x); }

// Pair exchange of registers k, k + 1 of one block (as in store_block): the even lane gets
// the 16 bytes of slots (0,0), (0,1) of its station pair, the odd lane (1,0), (1,1).
template <int ACC>
__device__ __forceinline__ void exchange_pair(const typename COp<ACC>::acc_t &re, const typename COp<ACC>::acc_t &im,
                                              int k, int om, bool odd, uint32_t (&v)[4])
{
    // element copies first: a bit cast of a vector element subscript reads element 0 with
    // this compiler
    const uint32_t r0 = bits32(re[k]), r1 = bits32(re[k + 1]);
    const uint32_t m0 = bits32(im[k]), m1 = bits32(im[k + 1]);
    const uint32_t xr = (uint32_t)swap_pair_lanes(pair_send((int)r0, (int)r1, om));
    const uint32_t xm = (uint32_t)swap_pair_lanes(pair_send((int)m0, (int)m1, om));
    v[0] = odd ? xr : r0;
    v[1] = odd ? xm : m0;
    v[2] = odd ? r1 : xr;
    v[3] = odd ? m1 : xm;
}

// Store two horizontally adjacent 32x32 blocks (columns col0 .. col0 + 63) when there are
// two polarisations and no window sums: after the pair exchange of store_block, one lane
// swap between the blocks (lanes 32..63 of the left block with lanes 0..31 of the right
// one) leaves each register with one row of 64 consecutive inputs, 32 stations, so that
// every store instruction writes 1 KiB of consecutive baselines.
template <int ACC>
__device__ __forceinline__ void store_pair(void *out_ptr, int nin, int f, int row0, int col0, int lane,
                                           const typename COp<ACC>::acc_t &re1, const typename COp<ACC>::acc_t &im1,
                                           const typename COp<ACC>::acc_t &re2, const typename COp<ACC>::acc_t &im2)
{
    using val_t = typename std::conditional<ACC == ACC_I8, int, float>::type;
    using vec4_t = typename std::conditional<ACC == ACC_I8, i32x4v, f32x4>::type;
    if (row0 >= nin || col0 >= nin) return;
    const int64_t nbl = (int64_t)(nin / 2) * (nin / 2 + 1) / 2;
    const bool odd = lane & 1;
    const int om = odd_lane_mask(lane);
    const int j = col0 + lane, s2 = j >> 1;
#pragma unroll
    for (int k = 0; k < 16; k += 2) {
        // pair exchange in each block (as in store_block): the even lane gets slots (0,0),
        // (0,1) of its station pair, the odd lane (1,0), (1,1)
        uint32_t v[2][4];
        exchange_pair<ACC>(re1, im1, k, om, odd, v[0]);
        exchange_pair<ACC>(re2, im2, k, om, odd, v[1]);
        // after the swap v[0] holds row i and v[1] row i + 4, columns col0 + lane
#pragma unroll
        for (int c = 0; c < 4; ++c) lane_swap32(v[0][c], v[1][c]);
        const int i = row0 + 8 * (k >> 2) + (k & 3);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ih = i + 4 * h, s1 = ih >> 1;
            if (ih >= nin || j >= nin || s1 < s2) continue;
            const int64_t o = ((int64_t)f * nbl + (int64_t)s1 * (s1 + 1) / 2 + s2) * 8 + (odd ? 4 : 0);
            const vec4_t w = __builtin_bit_cast(vec4_t, (u32x4){v[h][0], v[h][1], v[h][2], v[h][3]});
            __builtin_nontemporal_store(w, (vec4_t *)((val_t *)out_ptr + o));
        }
    }
}

// ---------------------------------------------------------------- work walk

// Position of a workgroup in its work: the (channel, window) items blockIdx.x,
// blockIdx.x + gridDim.x, ... (window-major, so that concurrent workgroups read
// neighbouring channels of the same time rows), walked one time block at a time.  All
// fields are wave-uniform.
template <int TB>
struct Cursor {
    int64_t item;
    int blk, nblk, f, t0, t1;
    bool valid;

    __device__ __forceinline__ void set(const XJob &p, int64_t it)
    {
        item = it;
        blk = 0;
        valid = it < p.nitems;
        if (valid) {
            const int w = (int)(it / p.nchan);
            f = (int)(it - (int64_t)w * p.nchan);
            t0 = w * p.window;
            t1 = min(p.ntime, t0 + p.window);
            nblk = (t1 - t0 + TB - 1) / TB;
        } else {  // past the end: empty blocks
            f = 0;
            t0 = t1 = 0;
            nblk = 1;
        }
    }
    __device__ __forceinline__ void init(const XJob &p) { set(p, blockIdx.x); }
    __device__ __forceinline__ void next(const XJob &p)
    {
        if (++blk == nblk) set(p, item + p.grid);
    }
};

// Descriptor of the block the cursor points at: rows t0 + TB blk .. of channel f; rows past
// the window (and everything past the last item) read as zero.
template <int TB>
__device__ __forceinline__ i32x4s block_rsrc(const XJob &p, const Cursor<TB> &c, uint64_t row_stride)
{
    const int r0 = c.t0 + c.blk * TB;
    const int nrows = max(0, min(TB, c.t1 - r0));
    const uint64_t base = (uint64_t)p.in + ((uint64_t)r0 * p.nchan + c.f) * (uint64_t)p.nin * 2;
    const uint32_t nrec = nrows ? (uint32_t)((nrows - 1) * row_stride + (uint64_t)p.nin * 2) : 0u;
    i32x4s r;
    r[0] = __builtin_amdgcn_readfirstlane((int)(uint32_t)base);
    r[1] = __builtin_amdgcn_readfirstlane((int)((uint32_t)(base >> 32) & 0xFFFFu));
    r[2] = __builtin_amdgcn_readfirstlane((int)nrec);
    r[3] = 0x00020000;
    return r;
}

// ---------------------------------------------------------------- wave work lists

// The 36 blocks of the triangle over eight waves, two per SIMD (waves w and w + 4 share a
// SIMD, so each SIMD carries nine blocks of MFMA work):
//   waves 0..3: the diagonal 2x2 triangle of block rows {2i, 2i+1} plus a two-block strip
//               that reuses two of its fragments: row 2 / 3 x columns {0,1} (i = 0, 1),
//               row 6 / 7 x columns {4,5} (i = 2, 3);
//   waves 4..7: the off-diagonal 2x2 squares rows {4,5} / {6,7} x columns {0,1} / {2,3}.
// F: block rows of the fragments a wave reads; BR/BC: per block, the fragment (index into
// F) of its rows and of its columns; ROT: fragments also needed in rotated form, the
// columns, or with ROWROT the rows (waves 1 and 3 have two row and four column fragments);
// PRE: the rotated column operands are read from LDS (fragments RC) instead.
// PAIR: blocks b whose right neighbour (same block row, next block column) is block b + 1,
// stored together; SINGLE: the block without a neighbour (-1: none).
template <int W>
struct Spec;
template <>
struct Spec<0> {
    static constexpr int NF = 3, NB = 5;
    static constexpr int F[4] = {0, 1, 2, 0}, BR[5] = {0, 1, 1, 2, 2}, BC[5] = {0, 0, 1, 0, 1};
    static constexpr bool ROT[4] = {true, true, false, false};
    static constexpr bool ROWROT = false, PRE = false;
    static constexpr int NPAIR = 2, PAIR[2] = {1, 3}, SINGLE = 0;
};
template <>
struct Spec<1> {
    static constexpr int NF = 4, NB = 5;
    static constexpr int F[4] = {2, 3, 0, 1}, BR[5] = {0, 1, 1, 1, 1}, BC[5] = {0, 0, 1, 2, 3};
    static constexpr bool ROT[4] = {true, true, false, false};
    static constexpr bool ROWROT = true, PRE = false;
    static constexpr int NPAIR = 2, PAIR[2] = {3, 1}, SINGLE = 0;
};
template <>
struct Spec<2> {
    static constexpr int NF = 3, NB = 5;
    static constexpr int F[4] = {4, 5, 6, 0}, BR[5] = {0, 1, 1, 2, 2}, BC[5] = {0, 0, 1, 0, 1};
    static constexpr bool ROT[4] = {true, true, false, false};
    static constexpr bool ROWROT = false, PRE = false;
    static constexpr int NPAIR = 2, PAIR[2] = {1, 3}, SINGLE = 0;
};
template <>
struct Spec<3> {
    static constexpr int NF = 4, NB = 5;
    static constexpr int F[4] = {6, 7, 4, 5}, BR[5] = {0, 1, 1, 1, 1}, BC[5] = {0, 0, 1, 2, 3};
    static constexpr bool ROT[4] = {true, true, false, false};
    static constexpr bool ROWROT = true, PRE = false;
    static constexpr int NPAIR = 2, PAIR[2] = {3, 1}, SINGLE = 0;
};
template <int I, int J>
struct SquareSpec {
    static constexpr int NF = 4, NB = 4;
    static constexpr int F[4] = {2 * I, 2 * I + 1, 2 * J, 2 * J + 1}, BR[5] = {0, 0, 1, 1, 0}, BC[5] = {2, 3, 2, 3, 0};
    static constexpr bool ROT[4] = {false, false, true, true};
    static constexpr bool ROWROT = false, PRE = false;
    static constexpr int NPAIR = 2, PAIR[2] = {0, 2}, SINGLE = -1;
};
template <>
struct Spec<4> : SquareSpec<2, 0> {};
template <>
struct Spec<5> : SquareSpec<2, 1> {};
template <>
struct Spec<6> : SquareSpec<3, 0> {};
template <>
struct Spec<7> : SquareSpec<3, 1> {};

constexpr int MAXB = 5;

template <int ACC>
struct AccSet {
    typename COp<ACC>::acc_t re[MAXB], im[MAXB];
};

// ---------------------------------------------------------------- kernel

// Position of the n-th fragment of wave W that is also needed rotated, and their count.
template <typename S>
constexpr int rot_index(int n)
{
    int c = 0;
    for (int x = 0; x < S::NF; ++x)
        if (S::ROT[x]) {
            if (c == n) return x;
            ++c;
        }
    return -1;
}
template <typename S>
constexpr int rot_count()
{
    int c = 0;
    for (int x = 0; x < S::NF; ++x) c += S::ROT[x] ? 1 : 0;
    return c;
}

// The 2 NB MFMAs of one K-step of wave W from its plain operand fragments A: the real
// parts first, each of the first ones followed by the rotation of one fragment (vector ALU
// work that runs while the matrix cores are busy), then the imaginary parts.  `early` (copy
// issue) runs after the first MFMA and `mid` (more vector work) after the second
// imaginary-part MFMA.  The scheduling barriers keep this order.
template <int ACC, typename S, typename Early, typename Mid>
__device__ __forceinline__ void mma_step(const Frag<COp<ACC>::FW> (&A)[S::NF], AccSet<ACC> &acc, Early &&early,
                                         Mid &&mid)
{
    if constexpr (S::PRE) {
        // rotated column operands staged in LDS: no rotation in registers
        static_for<S::NB>([&](auto B) __attribute__((always_inline)) {
            constexpr int b = decltype(B)::value;
            mma(acc.re[b], A[S::BR[b]], A[S::BC[b]]);
            if constexpr (b == 0) early();
            __builtin_amdgcn_sched_barrier(0);
        });
        static_for<S::NB>([&](auto B) __attribute__((always_inline)) {
            constexpr int b = decltype(B)::value;
            mma(acc.im[b], A[S::BR[b]], A[S::RC[b]]);
            if constexpr (b == 1) mid();
            __builtin_amdgcn_sched_barrier(0);
        });
        return;
    }
    constexpr int NROT = rot_count<S>();
    static_assert(NROT <= S::NB, "rotations ride on the real-part MFMAs");
    Frag<COp<ACC>::FW> Rt[S::NF];
    static_for<S::NB>([&](auto B) __attribute__((always_inline)) {
        constexpr int b = decltype(B)::value;
        mma(acc.re[b], A[S::BR[b]], A[S::BC[b]]);
        if constexpr (b == 0) early();
        if constexpr (b < NROT) {
            constexpr int x = rot_index<S>(b);
            Rt[x] = op_rot<ACC, !S::ROWROT>(A[x]);
        }
        __builtin_amdgcn_sched_barrier(0);
    });
    static_for<S::NB>([&](auto B) __attribute__((always_inline)) {
        constexpr int b = decltype(B)::value;
        if constexpr (S::ROWROT) mma(acc.im[b], Rt[S::BR[b]], A[S::BC[b]]);
        else mma(acc.im[b], A[S::BR[b]], Rt[S::BC[b]]);
        if constexpr (b == 1) mid();
        __builtin_amdgcn_sched_barrier(0);
    });
}

// Transposing reads of the raw fragments of work list S at K-step KSTEP (rows of ROWB bytes).
template <int ACC, typename S, int KSTEP, int ROWB = CROW>
__device__ __forceinline__ void read_step(const uint32_t (&lv)[4], Raw<ACC> (&r)[S::NF])
{
    static_for<S::NF>([&](auto X) __attribute__((always_inline)) {
        constexpr int x = decltype(X)::value;
        r[x] = read_frag<ACC, S::F[x], KSTEP, ROWB>(lv);
    });
}

// All K-steps of one block on raw operands, software pipelined: the reads of K-step k + 1
// are issued before the MFMAs of K-step k, so that a wave keeps its matrix core busy while
// the other wave of its SIMD waits at the barrier.  copy(k) issues the copies due at
// K-step k.
template <int ACC, typename S, int NKS, int ROWB = CROW, typename Copy, typename Mid, typename Pre>
__device__ __forceinline__ void block_raw(const uint32_t (&lv)[4], AccSet<ACC> &acc, Copy &&copy, Mid &&mid, Pre &&pre)
{
    Raw<ACC> ra[S::NF], rb[S::NF];
    read_step<ACC, S, 0, ROWB>(lv, ra);
    static_for<NKS>([&](auto K) __attribute__((always_inline)) {
        constexpr int k = decltype(K)::value;
        Raw<ACC>(&cur)[S::NF] = (k & 1) ? rb : ra;
        Raw<ACC>(&nxt)[S::NF] = (k & 1) ? ra : rb;
        pre(K);
        if constexpr (k + 1 < NKS) read_step<ACC, S, k + 1, ROWB>(lv, nxt);
        __builtin_amdgcn_sched_barrier(0);
        Frag<COp<ACC>::FW> A[S::NF];
        static_for<S::NF>([&](auto X) __attribute__((always_inline)) {
            constexpr int x = decltype(X)::value;
            A[x] = op_plain<ACC>(cur[x]);
        });
        mma_step<ACC, S>(A, acc, [&]() __attribute__((always_inline)) { copy(K); },
                         [&]() __attribute__((always_inline)) { mid(K); });
    });
}

// Stores of work list S.  Fragment rows F < 8 start at input row_base + 32 F, rows F >= 8
// (the column segment of a rectangle piece) at col_base + 32 (F - 8); the whole-channel
// kernel passes zero for both.
template <typename S>
__device__ __forceinline__ int frag_row0(int x, int row_base, int col_base)
{
    return S::F[x] >= 8 ? col_base + 32 * (S::F[x] - 8) : row_base + 32 * S::F[x];
}

template <int ACC, typename S>
__device__ __forceinline__ void store_all(const XJob &p, int f, int lane, AccSet<ACC> &acc, int row_base = 0,
                                          int col_base = 0)
{
    // Opaque copies: the validity masks of the stores depend only on the lane and the array
    // shape, and would otherwise be hoisted out of the channel loop as hundreds of live
    // scalar lane masks.
    int nin = p.nin, npol = p.npol, accumulate = p.accumulate, l = lane;
    asm volatile("" : "+s"(nin), "+s"(npol), "+s"(accumulate), "+v"(l));
    if (npol == 2 && !accumulate) {
        static_for<S::NPAIR>([&](auto P) __attribute__((always_inline)) {
            constexpr int b = S::PAIR[decltype(P)::value];
            static_assert(S::BR[b] == S::BR[b + 1] && S::F[S::BC[b + 1]] == S::F[S::BC[b]] + 1, "adjacent pair");
            store_pair<ACC>(p.out, nin, f, frag_row0<S>(S::BR[b], row_base, col_base),
                            frag_row0<S>(S::BC[b], row_base, col_base), l, acc.re[b], acc.im[b], acc.re[b + 1],
                            acc.im[b + 1]);
        });
        if constexpr (S::SINGLE >= 0) {
            constexpr int b = S::SINGLE;
            store_block<ACC>(p.out, nin, npol, accumulate, f, frag_row0<S>(S::BR[b], row_base, col_base),
                             frag_row0<S>(S::BC[b], row_base, col_base), l, acc.re[b], acc.im[b]);
        }
        return;
    }
    static_for<S::NB>([&](auto B) __attribute__((always_inline)) {
        constexpr int b = decltype(B)::value;
        store_block<ACC>(p.out, nin, npol, accumulate, f, frag_row0<S>(S::BR[b], row_base, col_base),
                         frag_row0<S>(S::BC[b], row_base, col_base), l, acc.re[b], acc.im[b]);
    });
}

extern __shared__ __attribute__((aligned(16))) uint8_t chan_lds[];

typedef __attribute__((address_space(3))) u32x4 lds_u4;

// Staged fp16 fragment of block row R for K-step KSTEP at lvf + 8192 KSTEP + 512 R (lvf:
// this lane's unit of the buffer, see run_wave).
template <typename S, int KSTEP>
__device__ __forceinline__ void read_staged(uint32_t lvf, Frag<4> (&A)[S::NF])
{
    static_for<S::NF>([&](auto X) __attribute__((always_inline)) {
        constexpr int x = decltype(X)::value;
        const u32x4 v = *(const lds_u4 *)(uintptr_t)(lvf + (uint32_t)(KSTEP * 8192 + S::F[x] * 512));
        A[x].w[0] = v[0]; A[x].w[1] = v[1]; A[x].w[2] = v[2]; A[x].w[3] = v[3];
    });
}

}  // namespace
}  // namespace xc
