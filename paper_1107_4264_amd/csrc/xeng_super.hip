// Super-tiled X-engine on the CDNA4 matrix cores (gfx950) for arrays of 272..2048 inputs
// (a multiple of 16; S = ceil(nin / 256) super-rows, the last one possibly partial): 4-bit
// complex samples on the int8 and fp8 paths, 8-bit samples on the int8 path.
//
// A channel's triangle (Eq. 4) is cut into S diagonal triangles of 256 inputs (the 36-block
// work lists of the whole-channel kernel) and S (S - 1) rectangles of 256 row inputs x 128
// column inputs (32 blocks, one 2x2 square per wave), run as two launches (one work list per
// kernel).  An item is (window, channel, piece); consecutive items go to workgroups of one
// XCD, so the pieces of a channel share their rows through its L2.  Per block of SP_TB time
// rows, the piece's input segments (256 row inputs and, for a rectangle, 128 column inputs)
// are copied into a raw LDS ring (one or two bytes per sample), then widened once into the
// layout the whole-channel kernel's int8 path reads (two bytes per sample, 16-byte chunks
// XOR-swizzled by row; 8-bit samples are only moved into that layout):
//   * int8: both components scaled by 8, exactly: 8 re = ((b & 0xF0) >> 1) | (b & 0x80) per
//     byte, and the same after moving the low nibble up; the products carry a factor 64,
//     divided out exactly before the stores.  In the rectangles the row segment, whose
//     operand is never negated, is scaled by 16 instead (16 re = b & 0xF0, a mask alone;
//     -8 becomes -128, which only the rotated column operand could not hold), so their
//     products carry 128; the planner keeps such jobs to windows of
//     floor((2^31 - 1) / (256 m^2)) samples;
//   * fp8: e4m3 pairs (all of -8..7 are exact), with the usual fp32 windows.
// The K-steps (software pipelined, Sec. 4.4's staging re-planned for gfx950), rotations and
// stores are those of the whole-channel kernel.  Variant bit 1 (rectangles): the widening
// also writes the column segment rotated to (-im, re) pairs, so that the imaginary
// products read their column operand from LDS: each column fragment is rotated once per
// block instead of once per K-step by each of the four waves that read it.

#include "xeng_chan_dev.h"

namespace xc {
namespace {

constexpr int SP_TB = 32;                  // time rows per block

// Raw geometry per sample format: BPS bytes per sample; AROW / BROW raw bytes per time row
// of the row / column segment; NA / NB copy instructions (1 KiB each) per block for them;
// DPW copies per wave per block (NA / 8 row copies and one column copy, the column copies
// repeated by two waves when NB = 4); UB raw bytes of one 16-byte widened chunk.
// Variant V (chosen by the autotuner): bit 0 keeps one block fewer in the raw ring; bit 1
// (rectangles, PRE) adds the rotated column segment to the widened rows.  CROW: widened
// bytes per time row (256 row inputs, 128 column inputs, with PRE their rotated copy);
// CONV: widened bytes per block.
template <int IN, int V = 0, int TRI = 1>
struct SGeo {
    static constexpr int BPS = IN == IN_CI8 ? 2 : 1;
    static constexpr int AROW = 256 * BPS, BROW = 128 * BPS;
    static constexpr int RAW = SP_TB * (AROW + BROW);
    static constexpr int RING = 4 - (V & 1);  // measured: 4 slots beat 3, 5, 6 and 8 (4-bit, 1024 inputs)
    static constexpr bool PRE = TRI == 0 && (V & 2);
    static constexpr int CROW = PRE ? 1024 : 768;
    static constexpr int CONV = SP_TB * CROW;
    static constexpr int LDS = RING * RAW + 2 * CONV;
    static constexpr int NA = SP_TB * AROW / 1024, NB = SP_TB * BROW / 1024;
    static constexpr int DPW = NA / 8 + 1;
    static constexpr int UB = 8 * BPS;
    static_assert(NA % 8 == 0 && 8 % NB == 0 && LDS <= 160 * 1024, "copy split and LDS budget");
};

// Rectangle pieces: wave W takes block rows {2 (W/2), 2 (W/2) + 1} and the column blocks
// {2 (W%2), 2 (W%2) + 1} of the column segment, stored as fragment rows 8..11.
template <int W>
struct RectSpec : SquareSpec<(W >> 1), 4 + (W & 1)> {};

// The same with the rotated column operands read from LDS: fragment rows 12..15 hold the
// column segment's block rows 0..3 as (-im, re) pairs.
template <int W>
struct RectRotSpec {
    static constexpr int I = W >> 1, J = W & 1;
    static constexpr int NF = 6, NB = 4;
    static constexpr int F[6] = {2 * I, 2 * I + 1, 8 + 2 * J, 9 + 2 * J, 12 + 2 * J, 13 + 2 * J};
    static constexpr int BR[5] = {0, 0, 1, 1, 0}, BC[5] = {2, 3, 2, 3, 0}, RC[5] = {4, 5, 4, 5, 0};
    static constexpr bool ROT[6] = {false, false, false, false, false, false};
    static constexpr bool ROWROT = false, PRE = true;
    static constexpr int NPAIR = 2, PAIR[2] = {0, 2}, SINGLE = -1;
};

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
    // n blocks at a time (the later ones may lie past the item's last block)
    __device__ __forceinline__ void next_n(const XJob &p, int n)
    {
        blk += n;
        if (blk >= nblk) set(p, step + 1);
    }
};

// Byte address of input 0 in the first row of the block the cursor points at.
template <typename C>
__device__ __forceinline__ uint64_t block_base(const XJob &p, const C &c, int bps)
{
    const int r0 = c.t0 + c.blk * SP_TB;
    return (uint64_t)p.in + (((uint64_t)r0 * p.nchan + c.f) * (uint64_t)p.nin) * bps;
}

// Descriptor of one input segment of the block the cursor points at, whose input 0 is at
// `bbase` (block_base): bytes `len` of each row from input `first`, bps bytes per sample;
// len 0 reads zeros.
template <typename C>
__device__ __forceinline__ i32x4s seg_rsrc(uint64_t bbase, const C &c, int first, int len, uint64_t row_stride,
                                           int bps)
{
    const int r0 = c.t0 + c.blk * SP_TB;
    const int nrows = len ? max(0, min(SP_TB, c.t1 - r0)) : 0;
    const uint64_t base = bbase + (uint64_t)(uint32_t)(first * bps);
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
// nibble spread to a byte mask by a third byte permute (selector byte 0 or 1 picks 0x00 or
// 0xFF; the arithmetic form (t << 8) - t is folded into a quarter-rate multiply).
__device__ __forceinline__ uint32_t nibbles_to_e4m3(uint32_t n)
{
    const uint32_t idx = n & 0x07070707u;
    const uint32_t pos = __builtin_amdgcn_perm(0x4E4C4A48u, 0x44403800u, idx);  // 0, 1, .., 7
    const uint32_t neg = __builtin_amdgcn_perm(0xB8C0C4C8u, 0xCACCCED0u, idx);  // -8, -7, .., -1
    const uint32_t t = (n >> 3) & 0x01010101u;
    const uint32_t m = __builtin_amdgcn_perm(0u, 0x0000FF00u, t);
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

// 16 x the samples (rectangles' row segment): the nibbles in the high half of each byte.
__device__ __forceinline__ void ci4x4_to_i8x16(uint32_t w, uint32_t &lo, uint32_t &hi)
{
    const uint32_t re = w & 0xF0F0F0F0u;
    const uint32_t im = (w << 4) & 0xF0F0F0F0u;
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

// -x of each byte (two's complement, no carries between bytes; -(-128) stays -128, which
// no operand here reaches)
__device__ __forceinline__ uint32_t neg_bytes(uint32_t x)
{
    const uint32_t n = ~x;
    return ((n & 0x7F7F7F7Fu) + 0x01010101u) ^ (n & 0x80808080u);
}

// The rotated forms, (-im, re) pairs, of ci4x4_to_i8x8 and ci4x4_to_e4m3x8.
__device__ __forceinline__ void ci4x4_to_i8x8_rot(uint32_t w, uint32_t &lo, uint32_t &hi)
{
    const uint32_t t = w & 0xF0F0F0F0u;
    const uint32_t re = (t >> 1) | (t & 0x80808080u);
    const uint32_t u = (w << 4) & 0xF0F0F0F0u;
    const uint32_t nim = neg_bytes((u >> 1) | (u & 0x80808080u));
    lo = __builtin_amdgcn_perm(re, nim, 0x05010400u);
    hi = __builtin_amdgcn_perm(re, nim, 0x07030602u);
}

__device__ __forceinline__ void ci4x4_to_e4m3x8_rot(uint32_t w, uint32_t &lo, uint32_t &hi)
{
    const uint32_t re = nibbles_to_e4m3((w >> 4) & 0x0F0F0F0Fu);
    const uint32_t nim = nibbles_to_e4m3(w & 0x0F0F0F0Fu) ^ 0x80808080u;
    lo = __builtin_amdgcn_perm(re, nim, 0x05010400u);
    hi = __builtin_amdgcn_perm(re, nim, 0x07030602u);
}

// int8 from 4-bit samples: the sums are 64 x the visibilities (triangles: both operands 8 x
// the samples) or 128 x (rectangles: 16 x and 8 x), exact shifts
template <int ACC, int IN, int TRI, typename S>
__device__ __forceinline__ void descale_store(const XJob &p, int f, int lane, AccSet<ACC> &acc, int row_base,
                                              int col_base)
{
    if constexpr (ACC == ACC_I8 && IN == IN_CI4) {
        constexpr int SH = TRI ? 6 : 7;
#pragma unroll
        for (int x = 0; x < S::NB; ++x) {
            acc.re[x] = acc.re[x] >> SH;
            acc.im[x] = acc.im[x] >> SH;
        }
    }
    store_all<ACC, S>(p, f, lane, acc, row_base, col_base);
}

// Widening kind of unit instruction M (see run_wave_super): row-segment units of a
// rectangle widen to 16 x the samples, the rest to 8 x, the fourth unit is rotated.
template <int TRI, int M>
constexpr int unit_kind_v = M < 2 ? (TRI ? 0 : 2) : (M == 2 ? 0 : 1);

template <int ACC, int IN, int TRI, int W, int V>
__device__ __forceinline__ void run_wave_super(const XJob &p, int lane)
{
    using Gs = SGeo<IN, V, TRI>;
    constexpr int RING = Gs::RING, DPW = Gs::DPW, NKS = SP_TB / COp<ACC>::KS;
    constexpr int NAW = Gs::NA / 8;    // row-segment copies per wave per block
    static_assert(NKS >= 1 && SP_TB % COp<ACC>::KS == 0, "whole K-steps per block");
    using acc_t = typename COp<ACC>::acc_t;
    constexpr bool PRE = Gs::PRE;
    constexpr int CROW_W = Gs::CROW, CONV = Gs::CONV;
    using S = typename std::conditional<TRI != 0, Spec<W>,
                                        typename std::conditional<PRE, RectRotSpec<W>, RectSpec<W>>::type>::type;
    constexpr int NUP = TRI ? 2 : 3;    // plain widening instructions per wave per block
    constexpr int NU = NUP + (PRE ? 1 : 0);  // and one of rotated column chunks with PRE
    const uint64_t row_stride = (uint64_t)p.nchan * p.nin * Gs::BPS;
    const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)chan_lds;
    const uint32_t conv0 = lds0 + RING * Gs::RAW;

    // copies (1 KiB each, lane l to LDS byte 16 l): row-segment instruction ia = 8 m + W
    // fills rows ia RA .. + RA - 1 (RA = 1024 / AROW), column-segment instruction W % NB the
    // rows (W % NB) RB .. + RB - 1 (waves W and W + 4 write the same bytes when NB = 4)
    constexpr int LA = Gs::AROW / 16, LB = Gs::BROW / 16;  // lanes per row
    const int ib = W % Gs::NB;
    uint32_t voff_a[NAW];
#pragma unroll
    for (int m = 0; m < NAW; ++m)
        voff_a[m] = (uint32_t)(((8 * m + W) * (1024 / Gs::AROW) + lane / LA) * row_stride + 16 * (lane % LA));
    const uint32_t voff_b = (uint32_t)((ib * (1024 / Gs::BROW) + lane / LB) * row_stride + 16 * (lane % LB));
    // The last super-row may be partial (nin not a multiple of 256): its chunks past the
    // last input read zeros (the rows below would otherwise hold the next channel).
    // the address of a block's input 0 advances by SP_TB rows per block within an item
    const uint64_t blk_bytes = (uint64_t)SP_TB * row_stride;
    auto issue = [&](const SCursor<TRI> &c, uint64_t bbase, int slot, int m) __attribute__((always_inline)) {
        const uint32_t sb = lds0 + slot * Gs::RAW;
        if (m < NAW) {
            const int va = min(Gs::AROW, (p.nin - c.seg_a) * Gs::BPS);  // valid bytes of a row
            const uint32_t vo = 16 * (lane % LA) < va ? voff_a[m] : COOB;
            dma16(seg_rsrc(bbase, c, c.seg_a, va, row_stride, Gs::BPS), sb + (8 * m + W) * 1024, vo);
        } else
            dma16(seg_rsrc(bbase, c, c.seg_b, TRI ? 0 : Gs::BROW, row_stride, Gs::BPS),
                  sb + SP_TB * Gs::AROW + ib * 1024, voff_b);
    };
    // dc.next with its block address kept up to date (recomputed only at a new item)
    auto advance = [&](SCursor<TRI> &c, uint64_t &bbase) __attribute__((always_inline)) {
        c.next(p);
        bbase = c.blk == 0 ? block_base(p, c, Gs::BPS) : bbase + blk_bytes;
    };

    // widening units, one 16-byte chunk of a widened row each: instructions m = 0, 1 of
    // wave W cover row-segment unit U = 512 m + 64 W + lane (row U / 32, chunk U % 32); in a
    // rectangle instruction 2 covers column-segment unit U = 64 W + lane (row U / 16, chunk
    // 32 + U % 16) and, with PRE, instruction 3 its rotated copy (chunk 48 + U % 16)
    static_assert(SP_TB * 32 == 1024 && SP_TB * 16 == 512, "units cover the block");
    uint32_t usrc[NU], udst[NU];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int U = 512 * m + 64 * W + lane;
        const int row = U >> 5, c = U & 31;
        usrc[m] = (uint32_t)(row * Gs::AROW + Gs::UB * c);
        udst[m] = (uint32_t)(row * CROW_W + 16 * (c ^ (4 * (row & 3))));
    }
#pragma unroll
    for (int m = 2; m < NU; ++m) {
        const int U = 64 * W + lane;
        const int row = U >> 4, r = U & 15, c = (m == 2 ? 32 : 48) + r;
        usrc[m] = (uint32_t)(SP_TB * Gs::AROW + row * Gs::BROW + Gs::UB * r);
        udst[m] = (uint32_t)(row * CROW_W + 16 * (c ^ (4 * (row & 3))));
    }
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) u32x2 lds_u2;
    // raw unit: 8 bytes of 4-bit samples, or 16 bytes of 8-bit samples (already int8 pairs)
    using raw_t = typename std::conditional<IN == IN_CI8, u32x4, u32x2>::type;
    // kind 0: 8 x the samples (int8) or e4m3; 1: the same rotated to (-im, re); 2: the
    // rectangles' row segment (16 x the samples on the int8 path)
    auto widen = [&](raw_t v, uint32_t dst, auto KindTag) __attribute__((always_inline)) {
        constexpr int KIND = decltype(KindTag)::value;
        constexpr bool ROTU = KIND == 1;
        if constexpr (IN == IN_CI8) {
            static_assert(ACC == ACC_I8, "8-bit samples: int8 path only");
            if constexpr (ROTU)
                *(lds_u4 *)(uintptr_t)dst = (u32x4){rotate_pairs<ACC_I8>(v[0]), rotate_pairs<ACC_I8>(v[1]),
                                                    rotate_pairs<ACC_I8>(v[2]), rotate_pairs<ACC_I8>(v[3])};
            else
                *(lds_u4 *)(uintptr_t)dst = v;
        } else {
            uint32_t o0, o1, o2, o3;
            if constexpr (ACC == ACC_I8 && KIND == 2) {
                ci4x4_to_i8x16(v[0], o0, o1);
                ci4x4_to_i8x16(v[1], o2, o3);
            } else if constexpr (ACC == ACC_I8 && ROTU) {
                ci4x4_to_i8x8_rot(v[0], o0, o1);
                ci4x4_to_i8x8_rot(v[1], o2, o3);
            } else if constexpr (ACC == ACC_I8) {
                ci4x4_to_i8x8(v[0], o0, o1);
                ci4x4_to_i8x8(v[1], o2, o3);
            } else if constexpr (ROTU) {
                ci4x4_to_e4m3x8_rot(v[0], o0, o1);
                ci4x4_to_e4m3x8_rot(v[1], o2, o3);
            } else {
                ci4x4_to_e4m3x8(v[0], o0, o1);
                ci4x4_to_e4m3x8(v[1], o2, o3);
            }
            *(lds_u4 *)(uintptr_t)dst = (u32x4){o0, o1, o2, o3};
        }
    };
    auto raw_read = [&](uint32_t a) __attribute__((always_inline)) {
        if constexpr (IN == IN_CI8) return (raw_t)(*(const lds_u4 *)(uintptr_t)a);
        else return (raw_t)(*(const lds_u2 *)(uintptr_t)a);
    };
    // the whole widening of one block (prologue)
    auto widen_block = [&](uint32_t src, uint32_t dst) __attribute__((always_inline)) {
        static_for<NU>([&](auto M) __attribute__((always_inline)) {
            constexpr int m = decltype(M)::value;
            widen(raw_read(src + usrc[m]), dst + udst[m], std::integral_constant<int, unit_kind_v<TRI, m>>{});
        });
    };

    uint32_t lb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) lb[q] = conv0 + lane_base<ACC, CROW_W>(lane, q);

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
    uint64_t dbase = block_base(p, dc, Gs::BPS);
#pragma unroll
    for (int d = 0; d < RING - 1; ++d) {
#pragma unroll
        for (int m = 0; m < DPW; ++m) issue(dc, dbase, d, m);
        advance(dc, dbase);
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
        const uint64_t ibase = dbase;
        const int dslot = slot == 0 ? RING - 1 : slot - 1;
        advance(dc, dbase);
        const uint32_t csrc = lds0 + (slot == RING - 1 ? 0 : slot + 1) * Gs::RAW;
        const uint32_t cdst = conv0 + (fb ^ 1) * CONV;
        uint32_t lv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) lv[q] = lb[q] + fb * CONV;
        // K-step k issues copy m (of the block RING - 1 ahead) when m NKS / DPW == k, and
        // widens unit u of the next block when u NKS / NU == k: the unit is read before the
        // MFMAs, widened and stored between them
        raw_t rr[NU];
        auto copy = [&](auto K) __attribute__((always_inline)) {
            static_for<DPW>([&](auto M) __attribute__((always_inline)) {
                if constexpr (decltype(M)::value * NKS / DPW == decltype(K)::value) issue(ic, ibase, dslot, decltype(M)::value);
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
                if constexpr (u * NKS / NU == decltype(K)::value)
                    widen(rr[u], cdst + udst[u], std::integral_constant<int, unit_kind_v<TRI, u>>{});
            });
        };
        block_raw<ACC, S, NKS, CROW_W>(lv, acc, copy, mid, pre);
        slot = slot == RING - 1 ? 0 : slot + 1;
        fb ^= 1;
        nc.next(p);

        if (++cc.blk == cc.nblk) {
            wait_vm<0>();
            ready = RING - 2;
            descale_store<ACC, IN, TRI, S>(p, cc.f, lane, acc, cc.seg_a, cc.seg_b);
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

template <int ACC, int IN, int TRI, int V>
__global__ __launch_bounds__(CT, 1) void xeng_super_kernel(XJob p)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    switch (wave) {
    case 0: run_wave_super<ACC, IN, TRI, 0, V>(p, lane); break;
    case 1: run_wave_super<ACC, IN, TRI, 1, V>(p, lane); break;
    case 2: run_wave_super<ACC, IN, TRI, 2, V>(p, lane); break;
    case 3: run_wave_super<ACC, IN, TRI, 3, V>(p, lane); break;
    case 4: run_wave_super<ACC, IN, TRI, 4, V>(p, lane); break;
    case 5: run_wave_super<ACC, IN, TRI, 5, V>(p, lane); break;
    case 6: run_wave_super<ACC, IN, TRI, 6, V>(p, lane); break;
    default: run_wave_super<ACC, IN, TRI, 7, V>(p, lane); break;
    }
}

template <int ACC, int IN, int TRI, int V>
int launch_super_kind(XJob job, int cus, hipStream_t stream)
{
    constexpr int LDS = SGeo<IN, V, TRI>::LDS;
    if (int e = allow_lds_on_device<xeng_super_kernel<ACC, IN, TRI, V>>(LDS)) return e;
    const int ns = job.ntile_side;
    job.nitems = (int64_t)job.nwindows * job.nchan * (TRI ? ns : ns * (ns - 1));
    job.grid = job.nitems < cus ? job.nitems : cus;
    if (job.grid <= 0) return 0;
    hipLaunchKernelGGL((xeng_super_kernel<ACC, IN, TRI, V>), dim3((unsigned)job.grid), dim3(CT), LDS, stream, job);
    return (int)hipGetLastError();
}

// Variant bit 0 applies to both launches, bit 1 (staged rotated column operands) to the
// rectangles.
template <int ACC, int IN>
int launch_super_pair(const XJob &job, int cus, hipStream_t stream)
{
    int e;
    switch (job.variant) {
    case 0: e = launch_super_kind<ACC, IN, 1, 0>(job, cus, stream); break;
    case 1: e = launch_super_kind<ACC, IN, 1, 1>(job, cus, stream); break;
    case 2: e = launch_super_kind<ACC, IN, 1, 0>(job, cus, stream); break;
    case 3: e = launch_super_kind<ACC, IN, 1, 1>(job, cus, stream); break;
    default: return (int)hipErrorInvalidValue;
    }
    if (e) return e;
    switch (job.variant) {
    case 0: return launch_super_kind<ACC, IN, 0, 0>(job, cus, stream);
    case 1: return launch_super_kind<ACC, IN, 0, 1>(job, cus, stream);
    case 2: return launch_super_kind<ACC, IN, 0, 2>(job, cus, stream);
    default: return launch_super_kind<ACC, IN, 0, 3>(job, cus, stream);
    }
}


// ---------------------------------------------------------------- fp6 e3m2 super-tiles
//
// 4-bit samples on fp6 e3m2 operands (three exponent bits of bias 3, two mantissa bits:
// every integer of [-8, 8] is exact) for the scaled f8f6f4 32x32x64 MFMA, at twice the
// fp8 rate.  A pre-pass converts each (channel, block of 32 samples, input) once into 48
// bytes: the 32 real parts as e3m2 codes (six words, code k at bits 6k .. 6k + 5, in
// sample order) and the 32 imaginary parts.  Lane-half h of a fragment reads half h of its
// input's codes, so an MFMA of two plain fragments sums re_i re_j + im_i im_j over
// the block (the real part of Eq. 4), and one whose row fragment has its lane halves
// exchanged and the second half negated, (im_i, -re_i), sums im_i re_j - re_i im_j (the
// imaginary part).  The halves of 32 consecutive inputs form a 1536-byte group: their 32
// real halves (24 bytes each), then their 32 imaginary halves, so that the lanes of a
// fragment read at 24-byte strides (fewer LDS bank conflicts than whole 48-byte units:
// 2-3 % faster).  Groups are stored [channel][block][input / 32], the inputs padded with
// zeros to whole super-rows and the last block's samples past ntime zero, so that a piece
// copies contiguous segments (12 KiB for 256 row inputs, 6 KiB for 128 column inputs)
// straight into LDS: the main kernel converts nothing.  Eight waves, two per SIMD, with
// 2 x 2 blocks each in a rectangle and four or five blocks of a SIMD's nine in a triangle;
// four blocks share a ring slot and its barrier, two slots (two blocks per slot: 8 %
// faster rectangles than one; four: another 1-3 %; an eight-block ring of single blocks
// was no faster than six).
// Measured and dropped: four waves with 2 x 4 blocks (their 256 accumulator registers
// spill), and the next block's fragments read during this block's MFMAs (no faster: the
// pieces are bound by LDS bandwidth, not by the reads' latency).

constexpr int F6_UNIT = 48;    // bytes per input per block
constexpr int F6_CT = 512;     // threads per workgroup: eight waves, two per SIMD
constexpr int F6_NSUB = 4;     // 32-sample blocks per LDS ring slot (one barrier each)
constexpr int F6_RING = F6_NSUB == 2 ? 3 : 2;  // slots in the LDS ring

// fp16 high bytes of four signed 4-bit values (one per byte, low nibble; the low bytes of
// these fp16 values are zero): byte tables of the values 0..7 and -8..-1 indexed by the
// low three bits, chosen by the sign bit of each nibble (spread to a byte mask by a third
// permute).
__device__ __forceinline__ uint32_t nibbles_to_f16hi(uint32_t n)
{
    const uint32_t idx = n & 0x07070707u;
    const uint32_t pos = __builtin_amdgcn_perm(0x47464544u, 0x42403C00u, idx);  // 0, 1, .., 7
    const uint32_t neg = __builtin_amdgcn_perm(0xBCC0C2C4u, 0xC5C6C7C8u, idx);  // -8, -7, .., -1
    const uint32_t t = (n >> 3) & 0x01010101u;
    const uint32_t m = __builtin_amdgcn_perm(0u, 0x0000FF00u, t);
    return (neg & m) | (pos & ~m);
}

// 32 fp16 values (two per word, sample order) -> six words of e3m2 codes (gfx950's packed
// conversion, scale 1; exact for the integers of [-8, 8]).
__device__ __forceinline__ void f16x32_to_e3m2(const uint32_t (&h)[16], uint32_t *w)
{
    typedef _Float16 h32 __attribute__((ext_vector_type(32)));
    typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));
    u32x16 hv;
#pragma unroll
    for (int k = 0; k < 16; ++k) hv[k] = h[k];
    const auto p = __builtin_amdgcn_cvt_scalef32_pk32_bf6_f16(__builtin_bit_cast(h32, hv), 1.0f);
#pragma unroll
    for (int k = 0; k < 6; ++k) w[k] = p[k];
}

// Pre-pass.  One thread: four consecutive inputs (one word of 4-bit samples per time row)
// of one block of 32 samples of one channel -> their real and imaginary halves.  Threads
// run over (channel, block, input group of four), input groups fastest: a wave reads 256
// consecutive bytes of each time row and writes 12 KiB of consecutive groups.
__global__ __launch_bounds__(256) void f6_pack_kernel(const uint8_t *__restrict__ in, uint8_t *__restrict__ work,
                                                      int nin, int nchan, int ntime, int ntb, int npad,
                                                      int64_t nthreads)
{
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= nthreads) return;  // whole waves: nthreads is a multiple of 64
    const int ng = npad >> 2;
    const int g = (int)(idx % ng);
    const int64_t q = idx / ng;
    const int tb = (int)(q % ntb);
    const int f = (int)(q / ntb);
    const int t0 = tb * SP_TB;
    const bool live = 4 * g < nin;
    uint32_t v[SP_TB];
#pragma unroll
    for (int t = 0; t < SP_TB; ++t)
        v[t] = (live && t0 + t < ntime) ? ((const uint32_t *)(in + ((size_t)(t0 + t) * nchan + f) * nin))[g] : 0u;
    uint32_t wr[24], wi[24];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        // byte e of each time row (input 4g + e), four rows per word: (re, im) nibbles
        const uint32_t sel = 0x0C0C0000u | ((uint32_t)(4 + e) << 8) | (uint32_t)e;
        uint32_t hr[16], hm[16];
#pragma unroll
        for (int qd = 0; qd < 8; ++qd) {
            const uint32_t *r = v + 4 * qd;
            const uint32_t u = __builtin_amdgcn_perm(__builtin_amdgcn_perm(r[3], r[2], sel),
                                                     __builtin_amdgcn_perm(r[1], r[0], sel), 0x05040100u);
            const uint32_t cr = nibbles_to_f16hi((u >> 4) & 0x0F0F0F0Fu);
            const uint32_t cm = nibbles_to_f16hi(u & 0x0F0F0F0Fu);
            hr[2 * qd] = __builtin_amdgcn_perm(0u, cr, 0x010C000Cu);
            hr[2 * qd + 1] = __builtin_amdgcn_perm(0u, cr, 0x030C020Cu);
            hm[2 * qd] = __builtin_amdgcn_perm(0u, cm, 0x010C000Cu);
            hm[2 * qd + 1] = __builtin_amdgcn_perm(0u, cm, 0x030C020Cu);
        }
        f16x32_to_e3m2(hr, wr + 6 * e);
        f16x32_to_e3m2(hm, wi + 6 * e);
    }
    // The wave's 256 inputs are eight groups of 32 (12 KiB); the lanes' halves pass through
    // LDS so that store k writes the wave's 16-byte chunks 64 k .. 64 k + 63 (1 KiB of
    // consecutive bytes).  A wave's 64 input groups never straddle a (channel, block):
    // npad / 4 is a multiple of 64.
    __shared__ u32x4 stage[4][64 * 12];
    const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
    // lane ln's inputs are 4 (ln % 8) .. + 3 of the wave's 32-input group ln / 8: their real
    // halves are chunks 96 (ln / 8) + 6 (ln % 8) + 0..5, their imaginary halves 48 further
    const int c0 = 96 * (ln >> 3) + 6 * (ln & 7);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        stage[wv][c0 + k] = (u32x4){wr[4 * k], wr[4 * k + 1], wr[4 * k + 2], wr[4 * k + 3]};
        stage[wv][c0 + 48 + k] = (u32x4){wi[4 * k], wi[4 * k + 1], wi[4 * k + 2], wi[4 * k + 3]};
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    u32x4 *o = (u32x4 *)(work + (((size_t)f * ntb + tb) * npad + 4 * (size_t)(g - ln)) * F6_UNIT);
#pragma unroll
    for (int k = 0; k < 12; ++k) o[64 * k + ln] = stage[wv][64 * k + ln];
}

// Ring slot per block: the row segment (256 inputs, 48 bytes each), and for a rectangle the
// column segment (128 inputs); NCOPY 1 KiB copies.
template <int TRI>
struct F6Geo {
    static constexpr int ROWB = 256 * F6_UNIT, COLB = TRI ? 0 : 128 * F6_UNIT;
    static constexpr int SUB = ROWB + COLB, SUBC = SUB / 1024;  // one block, its copies
    static constexpr int SLOT = F6_NSUB * SUB, NCOPY = F6_NSUB * SUBC, LDS = F6_RING * SLOT;
    static_assert(SUB % 1024 == 0 && LDS <= 160 * 1024, "whole copies and LDS budget");
};

// Triangle block i (0..8) of SIMD s: the nine blocks below the diagonal in block rows s and
// 7 - s, (s, 0 .. s) then (7 - s, 0 .. 7 - s).
constexpr int f6_tri_br(int s, int i) { return i <= s ? s : 7 - s; }
constexpr int f6_tri_bc(int s, int i) { return i <= s ? i : i - s - 1; }

// Work of wave W (waves W and W + 4 share a SIMD): NB blocks (BR, BC: block row in the row
// segment, block column in the column segment, which in a triangle is the same segment).
// Rectangles: block rows {2 (W / 2), + 1} x columns {2 (W % 2), + 1}; triangles: the first
// five of SIMD W % 4's nine blocks for W < 4, the last four for W >= 4.  DPW copies per
// block (copies W, W + 8, ..).
template <int TRI, int W>
struct F6Wave {
    static constexpr int NB = TRI ? (W < 4 ? 5 : 4) : 4;
    static constexpr int br(int b) { return TRI ? f6_tri_br(W & 3, (W < 4 ? 0 : 5) + b) : 2 * (W >> 1) + (b >> 1); }
    static constexpr int bc(int b) { return TRI ? f6_tri_bc(W & 3, (W < 4 ? 0 : 5) + b) : 2 * (W & 1) + (b & 1); }
    static constexpr bool uses_row(int r)
    {
        for (int b = 0; b < NB; ++b)
            if (br(b) == r) return true;
        return false;
    }
    static constexpr bool uses_col(int c)
    {
        for (int b = 0; b < NB; ++b)
            if (bc(b) == c) return true;
        return false;
    }
    // plain fragment f: f < 8 block row f of the row segment, f >= 8 block f - 8 of the
    // column segment (a triangle reads both roles from the row segment)
    static constexpr int plain_of_col(int c) { return TRI ? c : 8 + c; }
    static constexpr bool reads(int f) { return f < 8 ? (uses_row(f) || (TRI && uses_col(f))) : (!TRI && uses_col(f - 8)); }
    // greedy pairing for the stores: block b starts a pair with b + 1 (same row, next column)
    static constexpr int kind(int b)  // 2: pair start, 1: single, 0: second of a pair
    {
        int i = 0;
        while (i < NB) {
            const bool pr = i + 1 < NB && br(i) == br(i + 1) && bc(i + 1) == bc(i) + 1;
            if (i == b) return pr ? 2 : 1;
            if (pr && i + 1 == b) return 0;
            i += pr ? 2 : 1;
        }
        return 0;
    }
    static constexpr int DPW = (F6Geo<TRI>::NCOPY - W + 7) / 8;
};

struct F6Frag {
    uint32_t w[6];
};

typedef uint32_t f6_u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) f6_u32x2 f6_lds_u2;

__device__ __forceinline__ void read_f6(uint32_t a, F6Frag &x)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const f6_u32x2 v = *(const f6_lds_u2 *)(uintptr_t)(a + 8 * k);
        x.w[2 * k] = v[0];
        x.w[2 * k + 1] = v[1];
    }
}

// (re | im) -> (im | -re): the lane halves exchanged (one lane swap and one select per
// word), then the sign bits of the second half's codes flipped (nm: zero in lanes 0..31).
__device__ __forceinline__ void rotate_f6(const F6Frag &x, F6Frag &r, bool upper, const uint32_t (&nm)[3])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        uint32_t a = x.w[k], b = x.w[k];
        lane_swap32(a, b);  // a = (lo, lo), b = (hi, hi)
        r.w[k] = (upper ? a : b) ^ nm[k % 3];
    }
}

__device__ __forceinline__ void mma_f6(f32x16 &c, const F6Frag &a, const F6Frag &b)
{
    const i32x8 av = {(int)a.w[0], (int)a.w[1], (int)a.w[2], (int)a.w[3], (int)a.w[4], (int)a.w[5], 0, 0};
    const i32x8 bv = {(int)b.w[0], (int)b.w[1], (int)b.w[2], (int)b.w[3], (int)b.w[4], (int)b.w[5], 0, 0};
    // formats 3/3: fp6 e3m2 for both operands (six words each); E8M0 scales 2^0
    c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 3, 3, 0, 127, 0, 127);
}

// V (autotuner): 0 reads the rotated row fragments from LDS (the other half, sign bits
// flipped: 2 more fragment reads and 12 vector instructions per block; 8 % faster on the
// 4-bit 1024-input workload), 1 exchanges the lane halves of the plain ones in registers
// (36 vector instructions).
template <int TRI, int W, int V>
__device__ __forceinline__ void run_wave_f6(const XJob &p, int lane)
{
    using G = F6Geo<TRI>;
    using S = F6Wave<TRI, W>;
    constexpr int RING = F6_RING, DPW = S::DPW;
    static_assert((RING - 2) * DPW < 64, "vmcnt range");
    const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t *)chan_lds;
    const int ntb = (p.ntime + SP_TB - 1) / SP_TB;
    const int npad = 256 * p.ntile_side;
    // lane-half h reads the real (h = 0) or imaginary (h = 1) half of its input in the
    // 32-input group of the fragment's block
    const uint32_t lo = (uint32_t)(768 * (lane >> 5) + 24 * (lane & 31));
    const uint32_t lor = (uint32_t)(768 * (1 - (lane >> 5)) + 24 * (lane & 31));
    const bool upper = lane >= 32;
    const uint32_t hm = upper ? 0xFFFFFFFFu : 0u;
    const uint32_t nm[3] = {hm & 0x20820820u, hm & 0x08208208u, hm & 0x82082082u};  // sign bits 6k + 5

    // address of input 0 of the block the cursor points at; within an item it advances by
    // one block of groups per block (recomputed only at a new item)
    const uint64_t blk_bytes = (uint64_t)npad * F6_UNIT;
    auto block_base_f6 = [&](const SCursor<TRI> &c) __attribute__((always_inline)) {
        const int tb = (c.t0 / SP_TB) + c.blk;
        return (uint64_t)p.work + (uint64_t)((int64_t)c.f * ntb + tb) * blk_bytes;
    };
    auto advance = [&](SCursor<TRI> &c, uint64_t &bbase) __attribute__((always_inline)) {
        c.next_n(p, F6_NSUB);
        bbase = c.blk == 0 ? block_base_f6(c) : bbase + F6_NSUB * blk_bytes;
    };
    // descriptor of one segment of that block (nothing past the end)
    auto desc = [&](uint64_t bbase, bool valid, int first, int bytes) __attribute__((always_inline)) {
        const uint64_t base = bbase + (uint64_t)(uint32_t)(first * F6_UNIT);
        i32x4s r;
        r[0] = __builtin_amdgcn_readfirstlane((int)(uint32_t)base);
        r[1] = __builtin_amdgcn_readfirstlane((int)((uint32_t)(base >> 32) & 0xFFFFu));
        r[2] = valid ? bytes : 0;
        r[3] = 0x00020000;
        return r;
    };
    // the F6_NSUB blocks of a slot: the cursor's block and the following ones (zeros past
    // the item)
    auto issue = [&](const SCursor<TRI> &c, uint64_t bbase, int slot) __attribute__((always_inline)) {
        const uint32_t sb = lds0 + (uint32_t)(slot * G::SLOT);
        static_for<DPW>([&](auto M) __attribute__((always_inline)) {
            constexpr int k = W + 8 * decltype(M)::value;
            constexpr int h = k / G::SUBC, kk = k % G::SUBC;
            const bool v = c.valid && c.blk + h < c.nblk;
            const uint32_t dst = sb + (uint32_t)(h * G::SUB + 1024 * kk);
            if constexpr (kk < 12)
                dma16(desc(bbase + h * blk_bytes, v, c.seg_a, G::ROWB), dst, (uint32_t)(1024 * kk + 16 * lane));
            else
                dma16(desc(bbase + h * blk_bytes, v, TRI ? c.seg_a : c.seg_b, TRI ? G::ROWB : G::COLB), dst,
                      (uint32_t)(1024 * (kk - 12) + 16 * lane));
        });
    };

    f32x16 are[S::NB], aim[S::NB];
#pragma unroll
    for (int b = 0; b < S::NB; ++b) {
        are[b] = (f32x16){};
        aim[b] = (f32x16){};
    }
    F6Frag P[16], R[8];
    auto block = [&](int slot, int h) __attribute__((always_inline)) {
        const uint32_t sb = lds0 + (uint32_t)(slot * G::SLOT + h * G::SUB);
        static_for<16>([&](auto F) __attribute__((always_inline)) {
            constexpr int f = decltype(F)::value;
            if constexpr (S::reads(f))
                read_f6(sb + (f < 8 ? 0u : (uint32_t)G::ROWB) + 32 * F6_UNIT * (f & 7) + lo, P[f]);
        });
        static_for<8>([&](auto RB) __attribute__((always_inline)) {
            constexpr int r = decltype(RB)::value;
            if constexpr (S::uses_row(r)) {
                if constexpr (V & 1) {
                    rotate_f6(P[r], R[r], upper, nm);
                } else {
                    read_f6(sb + 32 * F6_UNIT * r + lor, R[r]);
#pragma unroll
                    for (int k = 0; k < 6; ++k) R[r].w[k] ^= nm[k % 3];
                }
            }
        });
        static_for<S::NB>([&](auto B) __attribute__((always_inline)) {
            constexpr int b = decltype(B)::value;
            constexpr int r = S::br(b), c = S::plain_of_col(S::bc(b));
            mma_f6(are[b], P[r], P[c]);
            mma_f6(aim[b], R[r], P[c]);
        });
    };
    auto store = [&](const SCursor<TRI> &c) __attribute__((always_inline)) {
        // opaque copies: keep the store masks from being hoisted out of the item loop
        int nin = p.nin, npol = p.npol, accumulate = p.accumulate, l = lane;
        asm volatile("" : "+s"(nin), "+s"(npol), "+s"(accumulate), "+v"(l));
        const int cb = TRI ? c.seg_a : c.seg_b;
        if (npol == 2 && !accumulate) {
            static_for<S::NB>([&](auto B) __attribute__((always_inline)) {
                constexpr int b = decltype(B)::value;
                if constexpr (S::kind(b) == 2)
                    store_pair<ACC_F8>(p.out, nin, c.f, c.seg_a + 32 * S::br(b), cb + 32 * S::bc(b), l, are[b], aim[b],
                                       are[b + 1], aim[b + 1]);
                else if constexpr (S::kind(b) == 1)
                    store_block<ACC_F8>(p.out, nin, npol, accumulate, c.f, c.seg_a + 32 * S::br(b),
                                        cb + 32 * S::bc(b), l, are[b], aim[b]);
            });
        } else {
            static_for<S::NB>([&](auto B) __attribute__((always_inline)) {
                constexpr int b = decltype(B)::value;
                store_block<ACC_F8>(p.out, nin, npol, accumulate, c.f, c.seg_a + 32 * S::br(b), cb + 32 * S::bc(b),
                                    l, are[b], aim[b]);
            });
        }
    };

    SCursor<TRI> dc, cc;
    dc.init(p);
    cc.init(p);
    uint64_t dbase = block_base_f6(dc);
#pragma unroll
    for (int d = 0; d < RING - 1; ++d) {
        issue(dc, dbase, d);
        advance(dc, dbase);
    }
    wait_vm<(RING - 2) * DPW>();
    int slot = 0, ready = 1;
    // items, each a loop over its blocks two at a time (one ring slot; past the item's last
    // block the slot holds zeros), then its stores.  A slot: its copies complete (own, then
    // everyone's: the barrier also means that every wave has issued the MFMAs of the
    // previous slot, so that slot is free); the copy of slot + RING - 1 into it; this
    // slot's fragments and MFMAs.
    while (cc.valid) {
        do {
            if (ready == 0) wait_vm<(RING - 2) * DPW>();
            else --ready;
            __syncthreads();
            issue(dc, dbase, slot == 0 ? RING - 1 : slot - 1);
            advance(dc, dbase);
            static_for<F6_NSUB>([&](auto H) __attribute__((always_inline)) { block(slot, decltype(H)::value); });
            slot = slot == RING - 1 ? 0 : slot + 1;
        } while ((cc.blk += F6_NSUB) < cc.nblk);
        wait_vm<0>();
        ready = RING - 1;
        store(cc);
#pragma unroll
        for (int b = 0; b < S::NB; ++b) {
            are[b] = (f32x16){};
            aim[b] = (f32x16){};
        }
        cc.set(p, cc.step + 1);
    }
    // no copy into LDS may outlive the workgroup
    wait_vm<0>();
}

template <int TRI, int V>
__global__ __launch_bounds__(F6_CT, 1) void xeng_super_f6_kernel(XJob p)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    switch (wave) {
    case 0: run_wave_f6<TRI, 0, V>(p, lane); break;
    case 1: run_wave_f6<TRI, 1, V>(p, lane); break;
    case 2: run_wave_f6<TRI, 2, V>(p, lane); break;
    case 3: run_wave_f6<TRI, 3, V>(p, lane); break;
    case 4: run_wave_f6<TRI, 4, V>(p, lane); break;
    case 5: run_wave_f6<TRI, 5, V>(p, lane); break;
    case 6: run_wave_f6<TRI, 6, V>(p, lane); break;
    default: run_wave_f6<TRI, 7, V>(p, lane); break;
    }
}

template <int TRI, int V>
int launch_super_f6_kind(XJob job, int cus, hipStream_t stream)
{
    constexpr int LDS = F6Geo<TRI>::LDS;
    if (int e = allow_lds_on_device<xeng_super_f6_kernel<TRI, V>>(LDS)) return e;
    const int ns = job.ntile_side;
    job.nitems = (int64_t)job.nwindows * job.nchan * (TRI ? ns : ns * (ns - 1));
    job.grid = job.nitems < cus ? job.nitems : cus;
    if (job.grid <= 0) return 0;
    hipLaunchKernelGGL((xeng_super_f6_kernel<TRI, V>), dim3((unsigned)job.grid), dim3(F6_CT), LDS, stream, job);
    return (int)hipGetLastError();
}

}  // namespace

// Both launches of a super-tiled job (triangles, then rectangles); each sets its own item
// count and grid (at most one workgroup per compute unit, `cus`).
int launch_super(const XJob &job, int acc, int in_fmt, int cus, hipStream_t stream)
{
    if (in_fmt == IN_CI4 && acc == ACC_F6) {
        // the pre-pass into the unit workspace, then triangles and rectangles
        if (!job.work || job.nin % 4 != 0) return (int)hipErrorInvalidValue;
        const int npad = 256 * job.ntile_side, ntb = (job.ntime + SP_TB - 1) / SP_TB;
        const int64_t nth = (int64_t)job.nchan * ntb * (npad / 4);
        if (nth > 0) {
            hipLaunchKernelGGL(f6_pack_kernel, dim3((unsigned)((nth + 255) / 256)), dim3(256), 0, stream,
                               (const uint8_t *)job.in, (uint8_t *)job.work, job.nin, job.nchan, job.ntime, ntb,
                               npad, nth);
            if (int e = (int)hipGetLastError()) return e;
        }
        if (job.variant == 1) {
            if (int e = launch_super_f6_kind<1, 1>(job, cus, stream)) return e;
            return launch_super_f6_kind<0, 1>(job, cus, stream);
        }
        if (job.variant != 0) return (int)hipErrorInvalidValue;
        if (int e = launch_super_f6_kind<1, 0>(job, cus, stream)) return e;
        return launch_super_f6_kind<0, 0>(job, cus, stream);
    }
    if (in_fmt == IN_CI4 && acc == ACC_I8) return launch_super_pair<ACC_I8, IN_CI4>(job, cus, stream);
    if (in_fmt == IN_CI4 && acc == ACC_F8) return launch_super_pair<ACC_F8, IN_CI4>(job, cus, stream);
    if (in_fmt == IN_CI8 && acc == ACC_I8) return launch_super_pair<ACC_I8, IN_CI8>(job, cus, stream);
    return (int)hipErrorInvalidValue;
}

}  // namespace xc
