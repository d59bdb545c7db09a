// Whole-channel X-engine on the CDNA4 matrix cores (gfx950) for arrays of up to 256
// complex 8-bit inputs.
//
// For such arrays one workgroup owns all the baselines of a channel (the whole lower
// triangle of Eq. 4 at 32x32 block granularity: 8 block rows, 36 blocks), so every input
// sample is read from HBM exactly once, as whole 512-byte rows of the [time][channel]
// [input] layout of Sec. 5.1; splitting a row between tiles costs half the bandwidth on
// this memory system.  The workgroup is persistent: it walks channels (and accumulation
// windows) blockIdx.x, blockIdx.x + gridDim.x, ... with one workgroup per compute unit.
//
// Data path for one block of time rows (64 for int8, 32 for fp16):
//   * the rows are copied from HBM straight into an LDS ring by buffer loads with the
//     LDS-destination bit (no registers involved), three blocks ahead of the block being
//     multiplied; the 16-byte chunks of a row are XOR-swizzled by the row index so that
//     the transposing reads below are free of bank conflicts;
//   * MFMA operands are read with ds_read_b64_tr_b16: one complex 8-bit sample is one
//     16-bit element, so the transposing read hands each lane four consecutive samples of
//     one input, which is the operand layout of a 32-row MFMA fragment (the fp16 path
//     converts each block once, exactly, into an fp16 operand buffer read with 16-byte
//     reads);
//   * the complex product is mapped to real MFMAs as in the tiled kernel: the real part is
//     the product of the (re, im) pair sequences and the imaginary part the product with
//     one side rotated to (-im, re) or (im, -re) (Eq. 5, four real MACs per complex MAC).
// Work split (register level of the hierarchy of Sec. 4.1): eight waves, two per SIMD,
// 36 blocks of 32x32 baselines: four lists of five blocks (a diagonal 2x2 triangle plus a
// two-block strip) and four off-diagonal 2x2 squares, so every SIMD carries nine blocks.
// Each K-step is software pipelined: the next K-step's operand reads are issued before the
// current MFMAs.

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
    static constexpr int TB = 32, RING = 5;
    static constexpr bool STAGE = true;
};
template <int ACC>
struct Geom {
    static constexpr int TB = ChanCfg<ACC>::TB, RING = ChanCfg<ACC>::RING;
    static constexpr bool STAGE = ChanCfg<ACC>::STAGE;
    static constexpr int BLK = TB * CROW;                   // raw bytes per block
    static constexpr int DPW = TB / 2 / (CT / 64);          // copies per wave per block
    static constexpr int QUADS = TB / 4;                    // 4-sample groups per block
    static constexpr int FBUF = STAGE ? QUADS * 256 * 16 : 0;  // staged operand bytes
    static constexpr int LDS = RING * BLK + 2 * FBUF;
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
// columns, or with ROWROT the rows (waves 1 and 3 have two row and four column fragments).
// PAIR: blocks b whose right neighbour (same block row, next block column) is block b + 1,
// stored together; SINGLE: the block without a neighbour (-1: none).
template <int W>
struct Spec;
template <>
struct Spec<0> {
    static constexpr int NF = 3, NB = 5;
    static constexpr int F[4] = {0, 1, 2, 0}, BR[5] = {0, 1, 1, 2, 2}, BC[5] = {0, 0, 1, 0, 1};
    static constexpr bool ROT[4] = {true, true, false, false};
    static constexpr bool ROWROT = false;
    static constexpr int NPAIR = 2, PAIR[2] = {1, 3}, SINGLE = 0;
};
template <>
struct Spec<1> {
    static constexpr int NF = 4, NB = 5;
    static constexpr int F[4] = {2, 3, 0, 1}, BR[5] = {0, 1, 1, 1, 1}, BC[5] = {0, 0, 1, 2, 3};
    static constexpr bool ROT[4] = {true, true, false, false};
    static constexpr bool ROWROT = true;
    static constexpr int NPAIR = 2, PAIR[2] = {3, 1}, SINGLE = 0;
};
template <>
struct Spec<2> {
    static constexpr int NF = 3, NB = 5;
    static constexpr int F[4] = {4, 5, 6, 0}, BR[5] = {0, 1, 1, 2, 2}, BC[5] = {0, 0, 1, 0, 1};
    static constexpr bool ROT[4] = {true, true, false, false};
    static constexpr bool ROWROT = false;
    static constexpr int NPAIR = 2, PAIR[2] = {1, 3}, SINGLE = 0;
};
template <>
struct Spec<3> {
    static constexpr int NF = 4, NB = 5;
    static constexpr int F[4] = {6, 7, 4, 5}, BR[5] = {0, 1, 1, 1, 1}, BC[5] = {0, 0, 1, 2, 3};
    static constexpr bool ROT[4] = {true, true, false, false};
    static constexpr bool ROWROT = true;
    static constexpr int NPAIR = 2, PAIR[2] = {3, 1}, SINGLE = 0;
};
template <int I, int J>
struct SquareSpec {
    static constexpr int NF = 4, NB = 4;
    static constexpr int F[4] = {2 * I, 2 * I + 1, 2 * J, 2 * J + 1}, BR[5] = {0, 0, 1, 1, 0}, BC[5] = {2, 3, 2, 3, 0};
    static constexpr bool ROT[4] = {false, false, true, true};
    static constexpr bool ROWROT = false;
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

template <int ACC, int W>
__device__ __forceinline__ void run_wave(const XJob &p, int lane)
{
    using O = COp<ACC>;
    using G = Geom<ACC>;
    constexpr int TB = G::TB, RING = G::RING, DPW = G::DPW;
    constexpr int NKS = TB / O::KS;
    const uint64_t row_stride = (uint64_t)p.nchan * p.nin * 2;
    const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)chan_lds;

    // Copies: instruction m of this wave fills rows 2 DPW W + 2m + lane / 32, physical chunk
    // lane % 32, which holds logical chunk (lane % 32) ^ 4 (row & 3).
    uint32_t voff[DPW];
    const int nchunk = (p.nin * 2 + 15) / 16;
#pragma unroll
    for (int m = 0; m < DPW; ++m) {
        const int row = 2 * DPW * W + 2 * m + (lane >> 5);
        const int c = (lane & 31) ^ (4 * (row & 3));
        voff[m] = c < nchunk ? (uint32_t)(row * row_stride + 16 * c) : COOB;
    }
    auto issue = [&](const Cursor<TB> &c, int slot) __attribute__((always_inline)) {
        const i32x4s rs = block_rsrc<TB>(p, c, row_stride);
        const uint32_t dst = lds0 + slot * G::BLK + 2 * DPW * W * CROW;
#pragma unroll
        for (int m = 0; m < DPW; ++m) dma16(rs, dst + 2 * m * CROW, voff[m]);
    };
    // The copies of one block spread over the K-steps of the block being multiplied:
    // instruction m at K-step m NKS / DPW, among the MFMAs (all of them leaving the barrier
    // at once would queue behind each other).
    auto copy_at = [&](auto K, const i32x4s &rs, uint32_t dst) __attribute__((always_inline)) {
        constexpr int k = decltype(K)::value;
        static_for<DPW>([&](auto M) __attribute__((always_inline)) {
            constexpr int m = decltype(M)::value;
            if constexpr (m * NKS / DPW == k) dma16(rs, dst + 2 * m * CROW, voff[m]);
        });
    };

    AccSet<ACC> acc;
#pragma unroll
    for (int x = 0; x < MAXB; ++x) {
        acc.re[x] = (typename O::acc_t){};
        acc.im[x] = (typename O::acc_t){};
    }
    auto finish_item = [&](Cursor<TB> &cc) __attribute__((always_inline)) {
        store_all<ACC, Spec<W>>(p, cc.f, lane, acc);
#pragma unroll
        for (int x = 0; x < MAXB; ++x) {
            acc.re[x] = (typename O::acc_t){};
            acc.im[x] = (typename O::acc_t){};
        }
        cc.set(p, cc.item + p.grid);
    };

    Cursor<TB> dc, cc;
    dc.init(p);
    cc.init(p);
#pragma unroll
    for (int d = 0; d < RING - 1; ++d) {
        issue(dc, d);
        dc.next(p);
    }

    if constexpr (!G::STAGE) {
        uint32_t lb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) lb[q] = lds0 + lane_base<ACC>(lane, q);
        int slot = 0;
        int ready = 0;  // blocks known complete without a wait (copied before the last stores)
        while (cc.valid) {
            // own copies of this block done (the later blocks may still be in flight), then
            // everyone's: the block is complete and the slot of the previous block is free.
            // After an epilogue the next RING - 1 blocks were awaited before its stores;
            // waiting on the counter would also wait for the stores.
            if (ready == 0) wait_vm<(RING - 2) * DPW>();
            else --ready;
            __syncthreads();
            const i32x4s rs = block_rsrc<TB>(p, dc, row_stride);
            const uint32_t dst = lds0 + (slot == 0 ? RING - 1 : slot - 1) * G::BLK + 2 * DPW * W * CROW;
            dc.next(p);

            uint32_t lv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) lv[q] = lb[q] + slot * G::BLK;
            block_raw<ACC, Spec<W>, NKS>(lv, acc, [&](auto K) __attribute__((always_inline)) { copy_at(K, rs, dst); },
                                         [](auto) {}, [](auto) {});
            slot = slot == RING - 1 ? 0 : slot + 1;

            if (++cc.blk == cc.nblk) {
                wait_vm<0>();
                ready = RING - 1;
                finish_item(cc);
            }
        }
    } else {
        // Staged operands: the block after the one being multiplied is converted into the
        // other buffer (unit of input i and samples 4q..4q+3 at 4096 q + 16 i), read from the
        // raw ring with transposing reads.  Only the waves with five blocks (0..3) convert:
        // the four-block waves share their SIMDs with them and are the ones the barriers
        // wait for.  Instruction u of converting wave W covers the 16-input group
        // ig = 4 (u % 4) + lane / 16 at sample group q = 2 W + u / 4; units u and u + 4 differ
        // by four sample rows.
        constexpr int CW = 4;                          // converting waves
        constexpr int UPW = 16 * G::QUADS / 4 / CW;    // conversion instructions per converting wave
        static_assert(UPW == 2 * NKS, "two conversion units per K-step");
        const uint32_t fb0 = lds0 + RING * G::BLK;
        uint32_t cin[4], cout[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ig = 4 * j + (lane >> 4), q = (UPW / 4) * (W < CW ? W : 0);
            const int k = (lane >> 2) & 3, a = lane & 3;
            const int row = 4 * q + k;
            const int chunk = (2 * ig + (a >> 1)) ^ (4 * k);
            cin[j] = (uint32_t)(row * CROW + 16 * chunk + 8 * (a & 1));
            cout[j] = (uint32_t)(4096 * q + 16 * (16 * ig + (lane & 15)));
        }
        auto convert_read = [&](int u, uint32_t src) __attribute__((always_inline)) {
            return __builtin_amdgcn_ds_read_tr16_b64_v4i16(
                (lds_s16x4 *)(uintptr_t)(src + cin[u & 3] + (uint32_t)((u >> 2) * 4 * CROW)));
        };
        auto convert_write = [&](int u, s16x4 v, uint32_t dst) __attribute__((always_inline)) {
            const uint2 w = __builtin_bit_cast(uint2, v);
            uint32_t o0, o1, o2, o3;
            f16_pairs(w.x, o0, o1);
            f16_pairs(w.y, o2, o3);
            *(lds_u4 *)(uintptr_t)(dst + cout[u & 3] + (uint32_t)((u >> 2) * 4096)) = (u32x4){o0, o1, o2, o3};
        };
        // this lane's unit of a staged fragment: sample group 2 KSTEP + lane / 32, input
        // 32 R + lane % 32
        const uint32_t lf = (uint32_t)(4096 * (lane >> 5) + 16 * (lane & 31));

        wait_vm<(RING - 2) * DPW>();
        __syncthreads();
        if constexpr (W < CW) {
#pragma unroll
            for (int u = 0; u < UPW; ++u) convert_write(u, convert_read(u, lds0), fb0);
        }
        int slot = 0, fb = 0;
        int ready = 0;
        while (cc.valid) {
            // the copy of the next block (own, then everyone's) and the conversion of this
            // one are complete; the raw slot of the previous block and the other operand
            // buffer are free
            if (ready == 0) wait_vm<(RING - 3) * DPW>();
            else --ready;
            __syncthreads();
            const i32x4s rs = block_rsrc<TB>(p, dc, row_stride);
            const uint32_t dst = lds0 + (slot == 0 ? RING - 1 : slot - 1) * G::BLK + 2 * DPW * W * CROW;
            dc.next(p);

            // multiply this block, software pipelined: at each K-step the reads of the next
            // K-step's fragments and of two conversion units of the next block are issued
            // before the MFMAs, and the units are converted and stored between them
            const uint32_t lvf = fb0 + fb * G::FBUF + lf;
            const uint32_t csrc = lds0 + (slot == RING - 1 ? 0 : slot + 1) * G::BLK, cdst = fb0 + (fb ^ 1) * G::FBUF;
            {
                using S = Spec<W>;
                Frag<4> fa[S::NF], fbk[S::NF];
                read_staged<S, 0>(lvf, fa);
                static_for<NKS>([&](auto K) __attribute__((always_inline)) {
                    constexpr int k = decltype(K)::value;
                    Frag<4>(&cur)[S::NF] = (k & 1) ? fbk : fa;
                    Frag<4>(&nxt)[S::NF] = (k & 1) ? fa : fbk;
                    s16x4 cv0, cv1;
                    if constexpr (W < CW) {
                        cv0 = convert_read(2 * k, csrc);
                        cv1 = convert_read(2 * k + 1, csrc);
                    }
                    if constexpr (k + 1 < NKS) read_staged<S, k + 1>(lvf, nxt);
                    __builtin_amdgcn_sched_barrier(0);
                    mma_step<ACC, S>(cur, acc, [&]() __attribute__((always_inline)) { copy_at(K, rs, dst); },
                                     [&]() __attribute__((always_inline)) {
                                         if constexpr (W < CW) {
                                             convert_write(2 * k, cv0, cdst);
                                             convert_write(2 * k + 1, cv1, cdst);
                                         }
                                     });
                });
            }
            slot = slot == RING - 1 ? 0 : slot + 1;
            fb ^= 1;

            if (++cc.blk == cc.nblk) {
                wait_vm<0>();
                ready = RING - 2;
                finish_item(cc);
            }
        }
    }
    // no copy into LDS may outlive the workgroup
    wait_vm<0>();
}

template <int ACC>
__global__ __launch_bounds__(CT, 1) void xeng_chan_kernel(XJob p)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // Waves w and w + 4 share a SIMD and the older one (w) wins its issue conflicts.  The
    // fp16 path gives it the five-block list and the conversion; the int8 path runs faster
    // with the four-block squares on the older waves.
    constexpr int X = ACC == ACC_I8 ? 4 : 0;
    switch (wave) {
    case 0: run_wave<ACC, 0 ^ X>(p, lane); break;
    case 1: run_wave<ACC, 1 ^ X>(p, lane); break;
    case 2: run_wave<ACC, 2 ^ X>(p, lane); break;
    case 3: run_wave<ACC, 3 ^ X>(p, lane); break;
    case 4: run_wave<ACC, 4 ^ X>(p, lane); break;
    case 5: run_wave<ACC, 5 ^ X>(p, lane); break;
    case 6: run_wave<ACC, 6 ^ X>(p, lane); break;
    default: run_wave<ACC, 7 ^ X>(p, lane); break;
    }
}


// ---------------------------------------------------------------- super-tiles

// Arrays of 256 S inputs (S >= 2) with 4-bit samples on the int8 matrix cores.  A
// channel's triangle is cut into S diagonal triangles of 256 inputs (the 36-block work
// lists above) and S (S - 1) rectangles of 256 row inputs x 128 column inputs (32 blocks,
// one 2x2 square per wave), run as two launches (one work list per kernel).  An item is
// (window, channel, piece), and the pieces of a channel go to workgroups of one XCD, whose
// L2 serves the rows they share.  Per block of
// SP_TB time rows, the piece's input segments (256 row inputs and, for a rectangle, 128
// column inputs) are copied into a raw ring (one byte per sample), then widened once into
// the layout the int8 path reads (two bytes per sample, 16-byte chunks XOR-swizzled by
// row), with both components scaled by 8, exactly: 8 re = ((b & 0xF0) >> 1) | (b & 0x80)
// per byte, and the same for the low nibble moved up.  The products carry a factor 64,
// divided out exactly before the stores (the planner keeps such jobs to one window of
// floor((2^31 - 1) / (128 m^2)) samples).

constexpr int SP_TB = 32, SP_RING = 5;
constexpr int SP_AROW = 256, SP_BROW = 128;          // raw bytes per time row of the two segments
constexpr int SP_RAW = SP_TB * (SP_AROW + SP_BROW);   // raw bytes per block
constexpr int SP_CROW = 768;                          // widened bytes per time row (384 inputs)
constexpr int SP_CONV = SP_TB * SP_CROW;              // widened bytes per block
constexpr int SP_LDS = SP_RING * SP_RAW + 2 * SP_CONV;
constexpr int SP_DPW = 2;                             // copies per wave per block

// Rectangle pieces: wave W takes block rows {2 (W/2), 2 (W/2) + 1} and the column blocks
// {2 (W%2), 2 (W%2) + 1} of the column segment, stored as fragment rows 8..11.
template <int W>
struct RectSpec : SquareSpec<(W >> 1), 4 + (W & 1)> {};

// Position in the work of a workgroup: item g = step * grid + pos, pos = (b % 8) grid / 8 +
// b / 8 when the grid is a multiple of 8 (consecutive items on one XCD); item
// g = (window * nchan + channel) * npiece + piece.  All fields are wave-uniform.
template <int TRI>
struct SCursor {
    int64_t step;
    int pos, blk, nblk, f, t0, t1;
    int seg_a, seg_b;  // first row input, first column input of the piece
    bool valid;

    __device__ __forceinline__ void set(const XJob &p, int64_t st)
    {
        step = st;
        blk = 0;
        const int64_t g = st * p.grid + pos;
        valid = g < p.nitems;
        if (valid) {
            const int ns = p.ntile_side, np = TRI ? ns : ns * (ns - 1);
            const int piece = (int)(g % np);
            const int64_t q = g / np;
            const int w = (int)(q / p.nchan);
            f = (int)(q - (int64_t)w * p.nchan);
            t0 = w * p.window;
            t1 = min(p.ntime, t0 + p.window);
            nblk = (t1 - t0 + SP_TB - 1) / SP_TB;
            if (TRI) {
                seg_a = seg_b = 256 * piece;
            } else {
                // piece = 2 (i (i - 1) / 2 + j) + h for super-rows j < i, half h
                const int h = piece & 1;
                int pr = piece >> 1, i = 1;
                while (pr >= i) {
                    pr -= i;
                    ++i;
                }
                seg_a = 256 * i;
                seg_b = 256 * pr + 128 * h;
            }
        } else {  // past the end: empty blocks
            f = 0;
            t0 = t1 = 0;
            nblk = 1;
            seg_a = seg_b = 0;
        }
    }
    __device__ __forceinline__ void init(const XJob &p)
    {
        const int b = blockIdx.x, G = (int)p.grid;
        pos = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
        set(p, 0);
    }
    __device__ __forceinline__ void next(const XJob &p)
    {
        if (++blk == nblk) set(p, step + 1);
    }
};

// Descriptor of one input segment of the block the cursor points at (bytes `len` of each
// row from input `first`); len 0 reads zeros.
template <typename C>
__device__ __forceinline__ i32x4s seg_rsrc(const XJob &p, const C &c, int first, int len, uint64_t row_stride)
{
    const int r0 = c.t0 + c.blk * SP_TB;
    const int nrows = len ? max(0, min(SP_TB, c.t1 - r0)) : 0;
    const uint64_t base = (uint64_t)p.in + ((uint64_t)r0 * p.nchan + c.f) * (uint64_t)p.nin + first;
    const uint32_t nrec = nrows ? (uint32_t)((nrows - 1) * row_stride + len) : 0u;
    i32x4s r;
    r[0] = __builtin_amdgcn_readfirstlane((int)(uint32_t)base);
    r[1] = __builtin_amdgcn_readfirstlane((int)((uint32_t)(base >> 32) & 0xFFFFu));
    r[2] = __builtin_amdgcn_readfirstlane((int)nrec);
    r[3] = 0x00020000;
    return r;
}

// Four 4-bit complex samples (one per byte: re high nibble, im low) -> two words of
// (8 re, 8 im) int8 pairs.
// e4m3 codes of four signed 4-bit values (one per byte, low nibble): two 8-entry byte
// tables (values 0..7 and -8..-1, indexed by the low three bits) and the sign bit of each
// nibble spread to a byte mask ((t << 8) - t is 0xFF per byte where t is 1, no carries).
__device__ __forceinline__ uint32_t nibbles_to_e4m3(uint32_t n)
{
    const uint32_t idx = n & 0x07070707u;
    const uint32_t pos = __builtin_amdgcn_perm(0x4E4C4A48u, 0x44403800u, idx);  // 0, 1, .., 7
    const uint32_t neg = __builtin_amdgcn_perm(0xB8C0C4C8u, 0xCACCCED0u, idx);  // -8, -7, .., -1
    const uint32_t t = (n >> 3) & 0x01010101u;
    const uint32_t m = (t << 8) - t;
    return (neg & m) | (pos & ~m);
}

// Four 4-bit complex samples (one per byte: re high nibble, im low) -> two words of
// (re, im) fp8 e4m3 pairs, exactly.
__device__ __forceinline__ void ci4x4_to_e4m3x8(uint32_t w, uint32_t &lo, uint32_t &hi)
{
    const uint32_t re = nibbles_to_e4m3((w >> 4) & 0x0F0F0F0Fu);
    const uint32_t im = nibbles_to_e4m3(w & 0x0F0F0F0Fu);
    lo = __builtin_amdgcn_perm(im, re, 0x05010400u);
    hi = __builtin_amdgcn_perm(im, re, 0x07030602u);
}

__device__ __forceinline__ void ci4x4_to_i8x8(uint32_t w, uint32_t &lo, uint32_t &hi)
{
    const uint32_t t = w & 0xF0F0F0F0u;
    const uint32_t re = (t >> 1) | (t & 0x80808080u);
    const uint32_t u = (w << 4) & 0xF0F0F0F0u;
    const uint32_t im = (u >> 1) | (u & 0x80808080u);
    lo = __builtin_amdgcn_perm(im, re, 0x05010400u);
    hi = __builtin_amdgcn_perm(im, re, 0x07030602u);
}

// int8: the operands are 8 x the samples, the sums 64 x the visibilities (exact shift)
template <int ACC, typename S>
__device__ __forceinline__ void descale_store(const XJob &p, int f, int lane, AccSet<ACC> &acc, int row_base,
                                              int col_base)
{
    if constexpr (ACC == ACC_I8) {
#pragma unroll
        for (int x = 0; x < S::NB; ++x) {
            acc.re[x] = acc.re[x] >> 6;
            acc.im[x] = acc.im[x] >> 6;
        }
    }
    store_all<ACC, S>(p, f, lane, acc, row_base, col_base);
}

template <int ACC, int TRI, int W>
__device__ __forceinline__ void run_wave_super(const XJob &p, int lane)
{
    constexpr int RING = SP_RING, DPW = SP_DPW, NKS = SP_TB / COp<ACC>::KS;
    static_assert(NKS >= 1 && SP_TB % COp<ACC>::KS == 0, "whole K-steps per block");
    using acc_t = typename COp<ACC>::acc_t;
    using S = typename std::conditional<TRI != 0, Spec<W>, RectSpec<W>>::type;
    constexpr int NU = TRI ? 2 : 3;    // widening instructions per wave per block
    constexpr int NCH = TRI ? 32 : 48; // 16-byte chunks of a widened row
    const uint64_t row_stride = (uint64_t)p.nchan * p.nin;
    const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)chan_lds;
    const uint32_t conv0 = lds0 + RING * SP_RAW;

    // copies: instruction A of wave W fills segment-A rows 4W .. 4W + 3 (16 chunks each),
    // instruction B of waves W and W + 4 the segment-B rows 8 (W % 4) .. + 7 (8 chunks each;
    // both waves write the same bytes)
    const int wb = W & 3;
    const uint32_t voff_a = (uint32_t)((4 * W + (lane >> 4)) * row_stride + 16 * (lane & 15));
    const uint32_t voff_b = (uint32_t)((8 * wb + (lane >> 3)) * row_stride + 16 * (lane & 7));
    auto issue = [&](const SCursor<TRI> &c, int slot, int m) __attribute__((always_inline)) {
        const uint32_t sb = lds0 + slot * SP_RAW;
        if (m == 0) dma16(seg_rsrc(p, c, c.seg_a, SP_AROW, row_stride), sb + 4 * W * SP_AROW, voff_a);
        else dma16(seg_rsrc(p, c, c.seg_b, TRI ? 0 : SP_BROW, row_stride), sb + SP_TB * SP_AROW + 8 * wb * SP_BROW,
                   voff_b);
    };

    // widening units: instruction m < NU of wave W covers unit U = 512 m + 64 W + lane, row
    // U / NCH, chunk U % NCH (chunks 0..31 from segment A, 32..47 from segment B)
    static_assert(NU * 512 == SP_TB * NCH, "units cover the block");
    uint32_t usrc[NU], udst[NU];
#pragma unroll
    for (int m = 0; m < NU; ++m) {
        const int U = 512 * m + 64 * W + lane;
        const int row = U / NCH, c = U - NCH * (U / NCH);
        usrc[m] = (uint32_t)(c < 32 ? row * SP_AROW + 8 * c : SP_TB * SP_AROW + row * SP_BROW + 8 * (c - 32));
        udst[m] = (uint32_t)(row * SP_CROW + 16 * (c ^ (4 * (row & 3))));
    }
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) u32x2 lds_u2;
    auto widen = [&](u32x2 v, uint32_t dst) __attribute__((always_inline)) {
        uint32_t o0, o1, o2, o3;
        if constexpr (ACC == ACC_I8) {
            ci4x4_to_i8x8(v[0], o0, o1);
            ci4x4_to_i8x8(v[1], o2, o3);
        } else {
            ci4x4_to_e4m3x8(v[0], o0, o1);
            ci4x4_to_e4m3x8(v[1], o2, o3);
        }
        *(lds_u4 *)(uintptr_t)dst = (u32x4){o0, o1, o2, o3};
    };
    auto raw_read = [&](uint32_t a) __attribute__((always_inline)) { return *(const lds_u2 *)(uintptr_t)a; };
    // the whole widening of one block (prologue)
    auto widen_block = [&](uint32_t src, uint32_t dst) __attribute__((always_inline)) {
#pragma unroll
        for (int m = 0; m < NU; ++m) widen(raw_read(src + usrc[m]), dst + udst[m]);
    };

    uint32_t lb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) lb[q] = conv0 + lane_base<ACC, SP_CROW>(lane, q);

    AccSet<ACC> acc;
#pragma unroll
    for (int x = 0; x < MAXB; ++x) {
        acc.re[x] = (acc_t){};
        acc.im[x] = (acc_t){};
    }

    SCursor<TRI> dc, nc, cc;
    dc.init(p);
    cc.init(p);
    nc.init(p);
#pragma unroll
    for (int d = 0; d < RING - 1; ++d) {
        issue(dc, d, 0);
        issue(dc, d, 1);
        dc.next(p);
    }
    nc.next(p);  // the block after cc's

    wait_vm<(RING - 2) * DPW>();
    __syncthreads();
    widen_block(lds0, conv0);
    int slot = 0, fb = 0, ready = 0;
    while (cc.valid) {
        // the copy of the next block (own, then everyone's) and the widening of this one
        // are complete; the raw slot of the previous block and the other buffer are free
        if (ready == 0) wait_vm<(RING - 3) * DPW>();
        else --ready;
        __syncthreads();
        const SCursor<TRI> ic = dc;
        const int dslot = slot == 0 ? RING - 1 : slot - 1;
        dc.next(p);
        const uint32_t csrc = lds0 + (slot == RING - 1 ? 0 : slot + 1) * SP_RAW;
        const uint32_t cdst = conv0 + (fb ^ 1) * SP_CONV;
        uint32_t lv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) lv[q] = lb[q] + fb * SP_CONV;
        // K-step k issues copy m (of the block RING - 1 ahead) when m NKS / DPW == k, and
        // widens unit u of the next block when u NKS / NU == k: the unit is read before the
        // MFMAs, widened and stored between them
        u32x2 rr[NU];
        auto copy = [&](auto K) __attribute__((always_inline)) {
            static_for<DPW>([&](auto M) __attribute__((always_inline)) {
                if constexpr (decltype(M)::value * NKS / DPW == decltype(K)::value) issue(ic, dslot, decltype(M)::value);
            });
        };
        auto pre = [&](auto K) __attribute__((always_inline)) {
            static_for<NU>([&](auto U) __attribute__((always_inline)) {
                constexpr int u = decltype(U)::value;
                if constexpr (u * NKS / NU == decltype(K)::value) rr[u] = raw_read(csrc + usrc[u]);
            });
        };
        auto mid = [&](auto K) __attribute__((always_inline)) {
            static_for<NU>([&](auto U) __attribute__((always_inline)) {
                constexpr int u = decltype(U)::value;
                if constexpr (u * NKS / NU == decltype(K)::value) widen(rr[u], cdst + udst[u]);
            });
        };
        block_raw<ACC, S, NKS, SP_CROW>(lv, acc, copy, mid, pre);
        slot = slot == RING - 1 ? 0 : slot + 1;
        fb ^= 1;
        nc.next(p);

        if (++cc.blk == cc.nblk) {
            wait_vm<0>();
            ready = RING - 2;
            descale_store<ACC, S>(p, cc.f, lane, acc, cc.seg_a, cc.seg_b);
#pragma unroll
            for (int x = 0; x < MAXB; ++x) {
                acc.re[x] = (acc_t){};
                acc.im[x] = (acc_t){};
            }
            cc.set(p, cc.step + 1);
        }
    }
    // no copy into LDS may outlive the workgroup
    wait_vm<0>();
}

template <int ACC, int TRI>
__global__ __launch_bounds__(CT, 1) void xeng_super_kernel(XJob p)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    switch (wave) {
    case 0: run_wave_super<ACC, TRI, 0>(p, lane); break;
    case 1: run_wave_super<ACC, TRI, 1>(p, lane); break;
    case 2: run_wave_super<ACC, TRI, 2>(p, lane); break;
    case 3: run_wave_super<ACC, TRI, 3>(p, lane); break;
    case 4: run_wave_super<ACC, TRI, 4>(p, lane); break;
    case 5: run_wave_super<ACC, TRI, 5>(p, lane); break;
    case 6: run_wave_super<ACC, TRI, 6>(p, lane); break;
    default: run_wave_super<ACC, TRI, 7>(p, lane); break;
    }
}

template <int ACC, int TRI>
int launch_super_kind(XJob job, int cus, hipStream_t stream)
{
    static int done = 0;
    if (!done) {
        const hipError_t e = hipFuncSetAttribute((const void *)xeng_super_kernel<ACC, TRI>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, SP_LDS);
        if (e != hipSuccess) return (int)e;
        done = 1;
    }
    const int ns = job.ntile_side;
    job.nitems = (int64_t)job.nwindows * job.nchan * (TRI ? ns : ns * (ns - 1));
    job.grid = job.nitems < cus ? job.nitems : cus;
    if (job.grid <= 0) return 0;
    hipLaunchKernelGGL((xeng_super_kernel<ACC, TRI>), dim3((unsigned)job.grid), dim3(CT), SP_LDS, stream, job);
    return (int)hipGetLastError();
}

// Dynamic LDS beyond the default limit, set once per kernel (one flag per path).
template <int ACC>
int allow_lds_chan()
{
    static int done = 0;
    if (!done) {
        const hipError_t e = hipFuncSetAttribute((const void *)xeng_chan_kernel<ACC>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, Geom<ACC>::LDS);
        if (e != hipSuccess) return (int)e;
        done = 1;
    }
    return 0;
}

template <int ACC>
int launch_chan_acc(const XJob &job, hipStream_t stream)
{
    auto k = xeng_chan_kernel<ACC>;
    if (int e = allow_lds_chan<ACC>()) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)job.grid), dim3(CT), Geom<ACC>::LDS, stream, job);
    return (int)hipGetLastError();
}

}  // namespace

// Both launches of a super-tiled job (triangles, then rectangles); each sets its own item
// count and grid (at most one workgroup per compute unit, `cus`).
int launch_super(const XJob &job, int acc, int cus, hipStream_t stream)
{
    if (acc == ACC_I8) {
        if (int e = launch_super_kind<ACC_I8, 1>(job, cus, stream)) return e;
        return launch_super_kind<ACC_I8, 0>(job, cus, stream);
    }
    if (acc == ACC_F8) {
        if (int e = launch_super_kind<ACC_F8, 1>(job, cus, stream)) return e;
        return launch_super_kind<ACC_F8, 0>(job, cus, stream);
    }
    return (int)hipErrorInvalidValue;
}

int launch_chan(const XJob &job, int acc, hipStream_t stream)
{
    if (job.grid <= 0) return 0;
    if (acc == ACC_I8) return launch_chan_acc<ACC_I8>(job, stream);
    if (acc == ACC_F16) return launch_chan_acc<ACC_F16>(job, stream);
    return (int)hipErrorInvalidValue;
}

}  // namespace xc
