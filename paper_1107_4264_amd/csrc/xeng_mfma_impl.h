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

#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "xeng.h"
#include "xeng_dev.h"

namespace xc {
namespace {

using namespace dev;

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
// fp32 operands: K = 2 per MFMA, one sample per lane-half.  A lane holds the real parts of
// G = 4 samples (words 0..3) and their imaginary parts (words 4..7): four K-steps of the
// fp32 MFMA each for the real and the imaginary components.
template <>
struct Op<ACC_F32M> {
    static constexpr int G = 4, WORDS = 8, TB = 16;
    using acc_t = f32x16;
};
// fp6 e3m2: 32x32x64 MFMAs like fp8, the 32 values of a lane packed into six words (one
// packed conversion from fp16).  The unit holds the plain operand (words 0..5, 6..7 zero)
// and the rotated one (-im, re) for the imaginary product (words 8..13): staged once, read
// as the column operand.
template <>
struct Op<ACC_F6> {
    static constexpr int G = 16, WORDS = 16, TB = 32;
    using acc_t = f32x16;
};



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


// ---------------------------------------------------------------- tile geometry

template <int ACC, int IN, int TILE>
struct Tile {
    using O = Op<ACC>;
    using acc_t = typename O::acc_t;
    static constexpr int G = O::G;
    static constexpr int TB = O::TB;
    static constexpr int WORDS = O::WORDS;
    static constexpr int PLANES = WORDS / 4;
    static constexpr int NTG = TB / G;                       // time groups per block
    static constexpr int BPC = InFmtT<IN>::BPC;
    static constexpr int CI = ((ACC == ACC_F8 || ACC == ACC_F6) && IN == IN_CI8) ? 4 : 8;  // inputs per load
    static constexpr int LW = CI * BPC / 4;                  // words per row load
    static constexpr int NT = NTG * (TILE / CI);             // staging tasks per side
    static constexpr int NB = TILE / 64;                     // 32x32 blocks per wave side
    static constexpr int PAD = 16;                           // bytes after each time group
    static constexpr int TG_BYTES = PLANES * TILE * 16 + PAD;
    static constexpr int SIDE_BYTES = NTG * TG_BYTES;
    static constexpr int LDS_BYTES = 2 * 2 * SIDE_BYTES;     // 2 buffers x 2 sides
    static constexpr int FULL = (1 << (NB * NB)) - 1;        // every block of the wave
    static constexpr int DIAG = NB == 2 ? 0xD : 1;           // blocks (0,0), (1,0), (1,1)
    static constexpr int DEPTH = (ACC == ACC_F16 || ACC == ACC_F32M) ? 3 : (ACC == ACC_I8 ? 2 : 1);  // blocks in flight
    static constexpr bool INTERLEAVE = false;                // convert between K-steps
    static_assert(2 * NT <= 256, "at most one staging task per thread");
    static_assert(TB % (2 * G) == 0, "time block holds whole K-steps");
};

// LDS layout of one side of one buffer: per time group a 16-byte unit per input (and per
// plane), then 16 bytes of padding.  The padding shifts consecutive time groups by four
// banks, so the stores of a staging wave (eight time groups x two input chunks per 16
// lanes) and the loads of an MFMA operand (sixteen consecutive inputs) hit 64 distinct
// banks; unit addresses differ by compile-time constants across K-steps and units.
template <int ACC, int IN, int TILE>
__device__ __forceinline__ uint32_t lds_off(int side, int tg, int plane, int row)
{
    using T = Tile<ACC, IN, TILE>;
    return (uint32_t)(side * T::SIDE_BYTES + tg * T::TG_BYTES + (plane * TILE + row) * 16);
}

// ---------------------------------------------------------------- staging

// Buffer descriptors over the rows of the time blocks of one channel: block k covers rows
// t_begin + k*TB .. min(t_begin + (k+1)*TB, t_end) - 1, each a run of nin samples.  Loads
// beyond a descriptor's size return zero in hardware, which pads the last block of a
// window and the tile beyond the last input without branches; blocks past the window get
// an empty descriptor.  All fields are wave-uniform and kept in scalar registers.
struct BlockRsrc {
    uint64_t base0;      // address of row t_begin of channel f
    uint64_t blk_bytes;  // TB rows
    uint32_t full_rec;   // bytes of a whole block
    uint32_t last_rec;   // bytes of the last block
    int nblk;

    __device__ __forceinline__ BlockRsrc(const XJob &p, int f, int t_begin, int t_end, int tb, int bpc)
    {
        const uint64_t row_stride = (uint64_t)p.nchan * p.nin * bpc;
        const uint64_t b0 = (uint64_t)p.in + (((uint64_t)t_begin * p.nchan + f) * p.nin) * bpc;
        // readfirstlane returns int: widen through uint32_t, or a low word >= 2^31 would
        // sign-extend into the high word of the address
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)b0);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(b0 >> 32));
        base0 = ((uint64_t)hi << 32) | (uint64_t)lo;
        blk_bytes = (uint64_t)tb * row_stride;
        nblk = __builtin_amdgcn_readfirstlane((t_end - t_begin + tb - 1) / tb);
        full_rec = __builtin_amdgcn_readfirstlane((uint32_t)(tb * row_stride));
        last_rec = __builtin_amdgcn_readfirstlane((uint32_t)((t_end - t_begin - (nblk - 1) * tb) * row_stride));
    }

    __device__ __forceinline__ __amdgpu_buffer_rsrc_t get(int blk) const
    {
        const uint32_t rec = blk < nblk - 1 ? full_rec : (blk == nblk - 1 ? last_rec : 0u);
        return __builtin_amdgcn_make_buffer_rsrc((void *)(base0 + (uint64_t)blk * blk_bytes), (short)0, (int)rec,
                                                 0x00020000);
    }
};

constexpr uint32_t OOB = 0xFFFFFFF0u;  // offset beyond any descriptor: the load returns zero

// Loads of one staging task: G rows (block rows row0 .. row0+G-1) of CI inputs from i0.
// MODE is the job's LoadMode: whole chunks (rows aligned to the chunk), 32-bit words (rows
// word aligned) or single bytes.
template <int ACC, int IN, int TILE, int MODE>
__device__ __forceinline__ void load_rows(__amdgpu_buffer_rsrc_t rs, uint32_t row_stride, int row0, int i0,
                                          int nin, uint32_t (&rows)[Tile<ACC, IN, TILE>::G][Tile<ACC, IN, TILE>::LW])
{
    using T = Tile<ACC, IN, TILE>;
#pragma unroll
    for (int u = 0; u < T::G; ++u) {
        const uint32_t roff = (uint32_t)(row0 + u) * row_stride;
        if constexpr (MODE == LOAD_VEC) {
            const uint32_t off = i0 < nin ? roff + (uint32_t)i0 * T::BPC : OOB;
            if constexpr (T::LW == 4) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
                rows[u][0] = v[0]; rows[u][1] = v[1]; rows[u][2] = v[2]; rows[u][3] = v[3];
            } else {
                const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
                rows[u][0] = v[0]; rows[u][1] = v[1];
            }
        } else if constexpr (MODE == LOAD_WORD) {
            // Word-aligned rows: a chunk that lies inside the row is one wide load (the HSA
            // runtime runs gfx9 and later in unaligned-access mode, so a 16-byte load needs
            // only 4-byte alignment); the chunk that runs past the last input goes word by
            // word, so that no load reaches beyond the row's last input.
            if (i0 + T::CI <= nin) {
                const uint32_t off = roff + (uint32_t)i0 * T::BPC;
                if constexpr (T::LW == 4) {
                    const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
                    rows[u][0] = v[0]; rows[u][1] = v[1]; rows[u][2] = v[2]; rows[u][3] = v[3];
                } else {
                    const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
                    rows[u][0] = v[0]; rows[u][1] = v[1];
                }
            } else {
                constexpr int PER_WORD = 4 / T::BPC;
#pragma unroll
                for (int k = 0; k < T::LW; ++k) {
                    const int ik = i0 + k * PER_WORD;
                    const uint32_t off = ik < nin ? roff + (uint32_t)ik * T::BPC : OOB;
                    rows[u][k] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < T::LW; ++k) {
                uint32_t w = 0;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int ib = i0 + (4 * k + c) / T::BPC;
                    const uint32_t off = ib < nin ? roff + (uint32_t)(i0 * T::BPC + 4 * k + c) : OOB;
                    w |= (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(rs, (int)off, 0, 0) << (8 * c);
                }
                rows[u][k] = w;
            }
        }
    }
}

// 16 words of (re, im) fp16 pairs -> the 32 values as fp6 e3m2 in six words (words 6, 7
// zero), by gfx950's packed conversion (scale 1).  Exact for integers of [-8, 8].
__device__ __forceinline__ void pack_fp6(const uint32_t (&h)[16], uint32_t *w)
{
    typedef _Float16 h32 __attribute__((ext_vector_type(32)));
    typedef uint32_t u32x16 __attribute__((ext_vector_type(16)));
    u32x16 hv;
#pragma unroll
    for (int k = 0; k < 16; ++k) hv[k] = h[k];
    const auto p = __builtin_amdgcn_cvt_scalef32_pk32_bf6_f16(__builtin_bit_cast(h32, hv), 1.0f);
#pragma unroll
    for (int k = 0; k < 6; ++k) w[k] = p[k];
    w[6] = w[7] = 0;
}

// Convert units E0 .. E1-1 (inputs of the chunk) of a task's rows to operand units and
// store them in LDS.
template <int ACC, int IN, int TILE, int E0 = 0, int E1 = Tile<ACC, IN, TILE>::CI>
__device__ __forceinline__ void stage_store(uint8_t *lds, int buf, int side, int tg, int chunk,
                                            const uint32_t (&rows)[Tile<ACC, IN, TILE>::G][Tile<ACC, IN, TILE>::LW])
{
    using T = Tile<ACC, IN, TILE>;
    uint8_t *base = lds + buf * 2 * T::SIDE_BYTES;
    if constexpr (ACC == ACC_F16 && IN == IN_CI8) {
        // unit of input e: word r = (fp16 re, fp16 im) of row r; row word k holds inputs
        // 2k and 2k+1
        static_assert(E0 % 2 == 0 && E1 % 2 == 0, "whole row words");
#pragma unroll
        for (int k = E0 / 2; k < E1 / 2; ++k) {
            uint32_t u0[4], u1[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) ci8x2_to_f16(rows[r][k], u0[r], u1[r]);
            const uint4 v0 = {u0[0], u0[1], u0[2], u0[3]};
            const uint4 v1 = {u1[0], u1[1], u1[2], u1[3]};
            *(uint4 *)(base + lds_off<ACC, IN, TILE>(side, tg, 0, chunk * T::CI + 2 * k)) = v0;
            *(uint4 *)(base + lds_off<ACC, IN, TILE>(side, tg, 0, chunk * T::CI + 2 * k + 1)) = v1;
        }
    } else {
#pragma unroll
        for (int e = E0; e < E1; ++e) {
            uint32_t u[T::WORDS];
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
            } else if constexpr (ACC == ACC_F6) {
                // the 16 rows' (re, im) as fp16 pairs, packed to fp6; then the rotated
                // (-im, re) pairs likewise
                uint32_t h[16];
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    int re, im;
                    pair_of<IN>(rows[m], e, re, im);
                    h[m] = f16_bits(re) | (f16_bits(im) << 16);
                }
                pack_fp6(h, u);
#pragma unroll
                for (int m = 0; m < 16; ++m) h[m] = rotate_pairs<ACC_F16>(h[m]);
                pack_fp6(h, u + 8);
            } else if constexpr (ACC == ACC_F32M) {
                // plane 0: real parts of the four rows, plane 1: imaginary parts
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    int re, im;
                    pair_of<IN>(rows[m], e, re, im);
                    u[m] = __builtin_bit_cast(uint32_t, (float)re);
                    u[4 + m] = __builtin_bit_cast(uint32_t, (float)im);
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
#pragma unroll
            for (int pl = 0; pl < T::PLANES; ++pl) {
                const uint4 v = {u[4 * pl], u[4 * pl + 1], u[4 * pl + 2], u[4 * pl + 3]};
                *(uint4 *)(base + lds_off<ACC, IN, TILE>(side, tg, pl, chunk * T::CI + e)) = v;
            }
        }
    }
}

// ---------------------------------------------------------------- MAC loop over one block

// Column operand of the imaginary product: (re, im) -> (-im, re) per sample.  Pairs sit in
// one word on the int8 / fp16 / fp8 paths; on the fp32 path the real and imaginary parts
// are separate words (0..3 and 4..7), so the rotation swaps the halves and negates one.
template <int ACC, int W>
__device__ __forceinline__ Frag<W> rotate_frag(const Frag<W> &b)
{
    Frag<W> c;
    if constexpr (ACC == ACC_F32M) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            c.w[k] = b.w[4 + k] ^ 0x80000000u;
            c.w[4 + k] = b.w[k];
        }
    } else if constexpr (ACC == ACC_F6) {
        // staged with the plain operand
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            c.w[k] = b.w[8 + k];
            c.w[8 + k] = 0;
        }
    } else {
#pragma unroll
        for (int k = 0; k < W; ++k) c.w[k] = rotate_pairs<ACC>(b.w[k]);
    }
    return c;
}

// acc += A^T B over one K-step: one MFMA (int8, fp16, fp8), or on the fp32 path eight
// 32x32x2 MFMAs (four samples per lane-half, real then imaginary components).
template <int ACC, typename AccT, int W>
__device__ __forceinline__ void mma_op(AccT &c, const Frag<W> &a, const Frag<W> &b)
{
    if constexpr (ACC == ACC_F32M) {
#pragma unroll
        for (int k = 0; k < 8; ++k)
            c = __builtin_amdgcn_mfma_f32_32x32x2f32(__builtin_bit_cast(float, a.w[k]),
                                                      __builtin_bit_cast(float, b.w[k]), c, 0, 0, 0);
    } else if constexpr (ACC == ACC_F6) {
        i32x8 av, bv;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            av[k] = (int)a.w[k];
            bv[k] = (int)b.w[k];
        }
        // formats 3/3 = fp6 e3m2 for both operands (six words each); E8M0 scales 2^0
        c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 3, 3, 0, 127, 0, 127);
    } else {
        mma(c, a, b);
    }
}

// One staged block: K-steps of 2G samples.  With two 32x32 blocks per wave side the wave
// computes blocks (0,0), (1,0), (1,1) and, unless it sits on the diagonal of a diagonal
// tile, block (0,1); the condition is wave-uniform, so the accumulators keep one register
// assignment and only a scalar branch guards the last pair of MFMAs.

// after(s) runs after the MFMAs of K-step s are issued: the caller converts and stores a
// share of the next block there, so that its VALU work issues while the MFMAs execute.
template <int ACC, int IN, int TILE>
__device__ __forceinline__ void read_frags(const uint8_t *base, int col_side, int wr, int wc, int r32, int tgk,
                                           Frag<Tile<ACC, IN, TILE>::WORDS> (&A)[Tile<ACC, IN, TILE>::NB],
                                           Frag<Tile<ACC, IN, TILE>::WORDS> (&B)[Tile<ACC, IN, TILE>::NB])
{
    using T = Tile<ACC, IN, TILE>;
    constexpr int NB = T::NB;
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
    }
}

// One staged block: K-steps of 2G samples, the operands of step s+1 read from LDS while
// the MFMAs of step s run.  With two 32x32 blocks per wave side the wave computes blocks
// (0,0), (1,0), (1,1) and, with DO01, block (0,1) (not on the diagonal of a diagonal
// tile).  after(s) runs once the MFMAs of step s are issued: the caller converts a share of
// the next block there, so that its VALU work issues while the MFMAs execute.
template <int ACC, int IN, int TILE, bool DO01, typename After>
__device__ __forceinline__ void mac_block(const uint8_t *base, int col_side, int wr, int wc, int lane,
                                          typename Tile<ACC, IN, TILE>::acc_t (&re)[Tile<ACC, IN, TILE>::NB][Tile<ACC, IN, TILE>::NB],
                                          typename Tile<ACC, IN, TILE>::acc_t (&im)[Tile<ACC, IN, TILE>::NB][Tile<ACC, IN, TILE>::NB],
                                          After &&after)
{
    using T = Tile<ACC, IN, TILE>;
    constexpr int NB = T::NB;
    constexpr int KSTEPS = T::NTG / 2;
    const int r32 = lane & 31, half = lane >> 5;
    Frag<T::WORDS> A[2][NB], B[2][NB];
    read_frags<ACC, IN, TILE>(base, col_side, wr, wc, r32, half, A[0], B[0]);
    static_for<KSTEPS>([&](auto S) __attribute__((always_inline)) {
        constexpr int s = decltype(S)::value;
        constexpr int cur = s & 1;
        if constexpr (s + 1 < KSTEPS)
            read_frags<ACC, IN, TILE>(base, col_side, wr, wc, r32, 2 * (s + 1) + half, A[cur ^ 1], B[cur ^ 1]);
        Frag<T::WORDS> C[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) C[b] = rotate_frag<ACC>(B[cur][b]);
        mma_op<ACC>(re[0][0], A[cur][0], B[cur][0]);
        mma_op<ACC>(im[0][0], A[cur][0], C[0]);
        if constexpr (NB == 2) {
            mma_op<ACC>(re[1][0], A[cur][1], B[cur][0]);
            mma_op<ACC>(im[1][0], A[cur][1], C[0]);
            mma_op<ACC>(re[1][1], A[cur][1], B[cur][1]);
            mma_op<ACC>(im[1][1], A[cur][1], C[1]);
            if constexpr (DO01) {
                mma_op<ACC>(re[0][1], A[cur][0], B[cur][1]);
                mma_op<ACC>(im[0][1], A[cur][0], C[1]);
            }
        }
        after(S);
    });
}

// ---------------------------------------------------------------- epilogue


template <int ACC, int IN, int TILE>
__device__ __forceinline__ void store_tile(const XJob &p, int f, int row0, int col0, int wr, int wc, int lane,
                                           int mask,
                                           typename Tile<ACC, IN, TILE>::acc_t (&re)[Tile<ACC, IN, TILE>::NB][Tile<ACC, IN, TILE>::NB],
                                           typename Tile<ACC, IN, TILE>::acc_t (&im)[Tile<ACC, IN, TILE>::NB][Tile<ACC, IN, TILE>::NB])
{
    using T = Tile<ACC, IN, TILE>;
    constexpr int NB = T::NB;
    using val_t = typename std::conditional<ACC == ACC_I8, int, float>::type;
    const int r32 = lane & 31, half = lane >> 5;
    const int npol = p.npol;
    const int64_t nbl = (int64_t)(p.nin / npol) * (p.nin / npol + 1) / 2;
    if (npol == 2 && !p.accumulate) {
        // Lanes 2k, 2k+1 hold columns q = 0, 1 of one station s2; registers k, k+1 hold
        // rows p = 0, 1 of one station s1.  After one exchange each lane stores 16 bytes:
        // the even lane the slots (0,0), (0,1), the odd lane the slots (1,0), (1,1).
        const bool odd = lane & 1;
        const int om = odd_lane_mask(lane);
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (!((mask >> (a * NB + b)) & 1)) continue;
                const int j = col0 + (wc * NB + b) * 32 + r32;
                const int s2 = j >> 1;
#pragma unroll
                for (int k = 0; k < 16; k += 2) {
                    const int i = row0 + (wr * NB + a) * 32 + 8 * (k >> 2) + 4 * half + (k & 3);
                    const int s1 = i >> 1;
                    const val_t r0 = (val_t)re[a][b][k], r1 = (val_t)re[a][b][k + 1];
                    const val_t m0 = (val_t)im[a][b][k], m1 = (val_t)im[a][b][k + 1];
                    const val_t xr = swap_pair_lanes(pair_send(r0, r1, om));
                    const val_t xm = swap_pair_lanes(pair_send(m0, m1, om));
                    if (i >= p.nin || j >= p.nin || s1 < s2) continue;
                    const int64_t o = ((int64_t)f * nbl + (int64_t)s1 * (s1 + 1) / 2 + s2) * 8 + (odd ? 4 : 0);
                    if constexpr (ACC == ACC_I8) {
                        const i32x4v v = odd ? (i32x4v){xr, xm, r1, m1} : (i32x4v){r0, m0, xr, xm};
                        __builtin_nontemporal_store(v, (i32x4v *)((int *)p.out + o));
                    } else {
                        const f32x4 v = odd ? (f32x4){xr, xm, r1, m1} : (f32x4){r0, m0, xr, xm};
                        __builtin_nontemporal_store(v, (f32x4 *)((float *)p.out + o));
                    }
                }
            }
        return;
    }
    const int npp = npol * npol;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (!((mask >> (a * NB + b)) & 1)) continue;
            const int j = col0 + (wc * NB + b) * 32 + r32;
            if (j >= p.nin) continue;
            const int s2 = j / npol, q = j - s2 * npol;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int i = row0 + (wr * NB + a) * 32 + 8 * (k >> 2) + 4 * half + (k & 3);
                if (i >= p.nin) continue;
                const int s1 = i / npol, pp = i - s1 * npol;
                if (s1 < s2) continue;
                const int64_t o = (((int64_t)f * nbl + (int64_t)s1 * (s1 + 1) / 2 + s2) * npp + pp * npol + q) * 2;
                if constexpr (ACC == ACC_I8) {
                    if (p.accumulate) {
                        unsigned long long *out = (unsigned long long *)p.out;
                        atomicAdd(&out[o], (unsigned long long)(long long)re[a][b][k]);
                        atomicAdd(&out[o + 1], (unsigned long long)(long long)im[a][b][k]);
                    } else {
                        *(int2 *)((int *)p.out + o) = make_int2(re[a][b][k], im[a][b][k]);
                    }
                } else {
                    if (p.accumulate) {
                        double *out = (double *)p.out;
                        atomicAdd(&out[o], (double)re[a][b][k]);
                        atomicAdd(&out[o + 1], (double)im[a][b][k]);
                    } else {
                        *(float2 *)((float *)p.out + o) = make_float2(re[a][b][k], im[a][b][k]);
                    }
                }
            }
        }
}

// ---------------------------------------------------------------- one work item

template <int ACC, int IN, int TILE, int MODE>
__device__ __forceinline__ void process_item(const XJob &p, int f, int g, int w, uint8_t *lds)
{
    using T = Tile<ACC, IN, TILE>;
    using acc_t = typename T::acc_t;
    constexpr int NB = T::NB;
    g = __builtin_amdgcn_readfirstlane(g);
    w = __builtin_amdgcn_readfirstlane(w);

    // Triangular tile index -> (bx, by), bx <= by (Sec. 4.2), exact integer fix-up.
    int by = (int)((sqrtf(8.0f * (float)g + 1.0f) - 1.0f) * 0.5f);
    while (by * (by + 1) / 2 > g) --by;
    while ((by + 1) * (by + 2) / 2 <= g) ++by;
    const int bx = g - by * (by + 1) / 2;
    const bool diag = (bx == by);
    const int row0 = by * TILE, col0 = bx * TILE;
    // item coordinates are wave-uniform: keep them (and the descriptors built from them)
    // in scalar registers
    f = __builtin_amdgcn_readfirstlane(f);
    const int t_begin = __builtin_amdgcn_readfirstlane(w * p.window);
    const int t_end = __builtin_amdgcn_readfirstlane(min(p.ntime, t_begin + p.window));
    const int nblk = (t_end - t_begin + T::TB - 1) / T::TB;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave >> 1, wc = wave & 1;

    // 32x32 blocks this wave computes (wave-uniform): skip blocks strictly above the
    // diagonal of a diagonal tile and blocks that start beyond the last input.
    int mask = 0;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int rbi = wr * NB + a, cbi = wc * NB + b;
            if (!(diag && rbi < cbi) && row0 + rbi * 32 < p.nin && col0 + cbi * 32 < p.nin)
                mask |= 1 << (a * NB + b);
        }
    mask = __builtin_amdgcn_readfirstlane(mask);

    acc_t re[NB][NB], im[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            re[a][b] = (acc_t){};
            im[a][b] = (acc_t){};
        }

    // Staging task of this thread: side, time group, input chunk.  A diagonal tile stages
    // one side; its spare threads repeat a task (same loads, same LDS values).
    const int nsides = diag ? 1 : 2;
    const int tix = tid % (nsides * T::NT);
    const int side = tix / T::NT;
    const int task = tix - side * T::NT;
    const int tg = task % T::NTG;
    const int chunk = task / T::NTG;
    const int i0 = (side == 0 ? row0 : col0) + chunk * T::CI;
    const uint32_t row_stride = (uint32_t)((int64_t)p.nchan * p.nin * T::BPC);
    using rows_t = uint32_t[T::G][T::LW];
    rows_t rows[T::DEPTH];

    // Loads past the last block read nothing (empty descriptor) and are issued anyway, so
    // the loop carries no branches between a load and the use of its registers.
    const BlockRsrc brs(p, f, t_begin, t_end, T::TB, T::BPC);
    auto load = [&](rows_t &rows, int blk) {
        load_rows<ACC, IN, TILE, MODE>(brs.get(blk), row_stride, tg * T::G, i0, p.nin, rows);
    };
    auto stage = [&](const rows_t &rows, int buf) { stage_store<ACC, IN, TILE>(lds, buf, side, tg, chunk, rows); };
    const int col_side = diag ? 0 : 1;
    // Any wave with a block to store computes (0,0), (1,0), (1,1), and (0,1) unless the
    // mask is the diagonal pattern; blocks of zero padding are computed but not stored.
    // The choice is made once per tile: the time loop exists in both forms, so the
    // accumulators never pass through a branch inside the loop.
    const bool active = mask != 0;
    constexpr int KSTEPS = T::NTG / 2;
    constexpr int UPS = T::CI / KSTEPS;  // units converted after each K-step

    auto run = [&](auto D) __attribute__((always_inline)) {
        constexpr bool DO01 = decltype(D)::value;
        // Multiply the block in LDS buffer `cur` while converting `rows` (the next block)
        // into buffer `cur ^ 1`, a share after each K-step (INTERLEAVE) or all at the end.
        auto step = [&](int cur, const rows_t &rows) __attribute__((always_inline)) {
            auto after = [&](auto S) __attribute__((always_inline)) {
                constexpr int s = decltype(S)::value;
                if constexpr (T::INTERLEAVE)
                    stage_store<ACC, IN, TILE, s * UPS, (s + 1) * UPS>(lds, cur ^ 1, side, tg, chunk, rows);
            };
            if (active)
                mac_block<ACC, IN, TILE, DO01>(lds + cur * 2 * T::SIDE_BYTES, col_side, wr, wc, lane, re, im, after);
            else if constexpr (T::INTERLEAVE)
                static_for<KSTEPS>(after);
            if constexpr (!T::INTERLEAVE) stage(rows, cur ^ 1);
        };
        // DEPTH register slots: while block b is multiplied, blocks b+1 .. b+DEPTH-1 are
        // in flight (block k lives in slot k % DEPTH); block b+1 is converted into the
        // other LDS buffer at the end of the step and block b+DEPTH is loaded into the
        // slot block b left.  One barrier per block.
        static_for<T::DEPTH>([&](auto S) __attribute__((always_inline)) { load(rows[decltype(S)::value], decltype(S)::value); });
        stage(rows[0], 0);
        __syncthreads();
        for (int blk = 0; blk < nblk; blk += T::DEPTH) {
            bool done = false;
            static_for<T::DEPTH>([&](auto S) __attribute__((always_inline)) {
                constexpr int k = decltype(S)::value;
                const int b = blk + k;
                if (done || b >= nblk) {
                    done = true;
                    return;
                }
                load(rows[k], b + T::DEPTH);
                step(b & 1, rows[(k + 1) % T::DEPTH]);
                __syncthreads();
            });
        }
    };
    if (mask != T::DIAG) run(std::true_type{});
    else run(std::false_type{});

    store_tile<ACC, IN, TILE>(p, f, row0, col0, wr, wc, lane, mask, re, im);
}

// ---------------------------------------------------------------- hardware-cache variant

// Operand unit of one input from its G raw samples s[u] (the low 16 bits of a CI8 sample,
// the low 8 bits of a CI4 sample): the same words the staged kernel writes to LDS.
template <int ACC, int IN, int G, int W>
__device__ __forceinline__ void unit_from_samples(const uint32_t (&s)[G], Frag<W> &o)
{
    auto pr = [&](int u, int &re, int &im) __attribute__((always_inline)) {
        if constexpr (IN == IN_CI8) {
            re = (int)(int8_t)(s[u] & 0xFF);
            im = (int)(int8_t)((s[u] >> 8) & 0xFF);
        } else {
            re = sext4((s[u] >> 4) & 0xF);
            im = sext4(s[u] & 0xF);
        }
    };
    if constexpr (ACC == ACC_I8) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if constexpr (IN == IN_CI8) {
                o.w[m] = (s[2 * m] & 0xFFFFu) | (s[2 * m + 1] << 16);
            } else {
                int r0, i0, r1, i1;
                pr(2 * m, r0, i0);
                pr(2 * m + 1, r1, i1);
                o.w[m] = (uint32_t)(r0 & 0xFF) | ((uint32_t)(i0 & 0xFF) << 8) | ((uint32_t)(r1 & 0xFF) << 16) |
                         ((uint32_t)(i1 & 0xFF) << 24);
            }
        }
    } else if constexpr (ACC == ACC_F16) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int re, im;
            pr(m, re, im);
            o.w[m] = f16_bits(re) | (f16_bits(im) << 16);
        }
    } else if constexpr (ACC == ACC_F32M) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int re, im;
            pr(m, re, im);
            o.w[m] = __builtin_bit_cast(uint32_t, (float)re);
            o.w[4 + m] = __builtin_bit_cast(uint32_t, (float)im);
        }
    } else if constexpr (ACC == ACC_F6) {
        uint32_t h[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            int re, im;
            pr(m, re, im);
            h[m] = f16_bits(re) | (f16_bits(im) << 16);
        }
        pack_fp6(h, o.w);
#pragma unroll
        for (int m = 0; m < 16; ++m) h[m] = rotate_pairs<ACC_F16>(h[m]);
        pack_fp6(h, o.w + 8);
    } else {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            int r0, i0, r1, i1;
            pr(2 * m, r0, i0);
            pr(2 * m + 1, r1, i1);
            const uint32_t w = __builtin_amdgcn_cvt_pk_fp8_f32((float)r0, (float)i0, 0, false);
            o.w[m] = __builtin_amdgcn_cvt_pk_fp8_f32((float)r1, (float)i1, w, true);
        }
    }
}

// One tile without the LDS stage: the hardware-managed cache of Sec. 4.3 against the
// software-managed one of Sec. 4.4.  Every wave loads its own operand fragments straight
// from memory, one sample of one input per lane and load (the 32 lanes of a half-wave read
// 32 consecutive inputs of one time row), and the waves and tiles that share inputs re-read
// them through the L1 and L2 caches.  Same arithmetic, diagonal skipping and epilogue as
// the staged tile; no barriers.  The next K-step's loads are issued before the current
// K-step's MFMAs.
template <int ACC, int IN, int TILE>
__device__ __forceinline__ void process_item_cache(const XJob &p, int f, int g, int w)
{
    using T = Tile<ACC, IN, TILE>;
    using acc_t = typename T::acc_t;
    constexpr int NB = T::NB, G = T::G, BPC = T::BPC;
    g = __builtin_amdgcn_readfirstlane(g);
    w = __builtin_amdgcn_readfirstlane(w);
    int by = (int)((sqrtf(8.0f * (float)g + 1.0f) - 1.0f) * 0.5f);
    while (by * (by + 1) / 2 > g) --by;
    while ((by + 1) * (by + 2) / 2 <= g) ++by;
    const int bx = g - by * (by + 1) / 2;
    const bool diag = (bx == by);
    const int row0 = by * TILE, col0 = bx * TILE;
    f = __builtin_amdgcn_readfirstlane(f);
    const int t_begin = __builtin_amdgcn_readfirstlane(w * p.window);
    const int t_end = __builtin_amdgcn_readfirstlane(min(p.ntime, t_begin + p.window));
    const int nsteps = (t_end - t_begin + 2 * G - 1) / (2 * G);

    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int wr = wave >> 1, wc = wave & 1;
    const int r32 = lane & 31, half = lane >> 5;
    int mask = 0;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int rbi = wr * NB + a, cbi = wc * NB + b;
            if (!(diag && rbi < cbi) && row0 + rbi * 32 < p.nin && col0 + cbi * 32 < p.nin) mask |= 1 << (a * NB + b);
        }
    mask = __builtin_amdgcn_readfirstlane(mask);

    acc_t re[NB][NB], im[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            re[a][b] = (acc_t){};
            im[a][b] = (acc_t){};
        }

    // Byte offset of each fragment's input within a time row (out of range: the load
    // returns zero) and of this lane's first sample row within a K-step.
    const uint32_t row_stride = (uint32_t)((int64_t)p.nchan * p.nin * BPC);
    const uint32_t chan_off = (uint32_t)((int64_t)f * p.nin * BPC);
    uint32_t ioff[2][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        const int i = row0 + (wr * NB + a) * 32 + r32, j = col0 + (wc * NB + a) * 32 + r32;
        ioff[0][a] = i < p.nin ? chan_off + (uint32_t)i * BPC : OOB;
        ioff[1][a] = j < p.nin ? chan_off + (uint32_t)j * BPC : OOB;
    }
    const uint32_t hoff = (uint32_t)(G * half) * row_stride;
    const uint64_t in0 = (uint64_t)p.in;

    using raw_t = uint32_t[2][NB][G];
    // K-step s: rows t_begin + 2G s .. of this channel; rows past the window read zero.
    auto load = [&](raw_t &r, int s) __attribute__((always_inline)) {
        const int t = t_begin + 2 * G * s;
        const int nrows = __builtin_amdgcn_readfirstlane(max(0, min(2 * G, t_end - t)));
        const uint64_t base = in0 + (uint64_t)t * row_stride;
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            (void *)base, (short)0, (int)((uint32_t)nrows * row_stride), 0x00020000);
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    const uint32_t off = ioff[sd][a] == OOB ? OOB : ioff[sd][a] + hoff + (uint32_t)u * row_stride;
                    if constexpr (IN == IN_CI8)
                        r[sd][a][u] = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)off, 0, 0);
                    else
                        r[sd][a][u] = __builtin_amdgcn_raw_buffer_load_b8(rs, (int)off, 0, 0);
                }
    };
    const bool active = mask != 0;
    auto run = [&](auto D) __attribute__((always_inline)) {
        constexpr bool DO01 = decltype(D)::value;
        raw_t raw[2];
        load(raw[0], 0);
        for (int s = 0; s < nsteps; s += 2) {
            static_for<2>([&](auto K) __attribute__((always_inline)) {
                constexpr int k = decltype(K)::value;
                if (s + k >= nsteps) return;
                load(raw[k ^ 1], s + k + 1);
                Frag<T::WORDS> A[NB], B[NB], C[NB];
#pragma unroll
                for (int a = 0; a < NB; ++a) {
                    unit_from_samples<ACC, IN, G>(raw[k][0][a], A[a]);
                    unit_from_samples<ACC, IN, G>(raw[k][1][a], B[a]);
                    C[a] = rotate_frag<ACC>(B[a]);
                }
                if (!active) return;
                mma_op<ACC>(re[0][0], A[0], B[0]);
                mma_op<ACC>(im[0][0], A[0], C[0]);
                if constexpr (NB == 2) {
                    mma_op<ACC>(re[1][0], A[1], B[0]);
                    mma_op<ACC>(im[1][0], A[1], C[0]);
                    mma_op<ACC>(re[1][1], A[1], B[1]);
                    mma_op<ACC>(im[1][1], A[1], C[1]);
                    if constexpr (DO01) {
                        mma_op<ACC>(re[0][1], A[0], B[1]);
                        mma_op<ACC>(im[0][1], A[0], C[1]);
                    }
                }
            });
        }
    };
    if (mask != T::DIAG) run(std::true_type{});
    else run(std::false_type{});
    store_tile<ACC, IN, TILE>(p, f, row0, col0, wr, wc, lane, mask, re, im);
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

extern __shared__ __attribute__((aligned(16))) uint8_t dyn_lds[];

template <int ACC, int IN, int TILE, int MODE>
__global__ __launch_bounds__(NTHREADS, 2) void xeng_mfma_kernel(XJob p)
{
    uint8_t *lds = dyn_lds;
    int f, g, w;
    if (!decode_item(p, p.block0 + blockIdx.x, f, g, w)) return;
    process_item<ACC, IN, TILE, MODE>(p, f, g, w, lds);
}

// The tiled kernel without LDS (one work item per workgroup).
template <int ACC, int IN, int TILE>
__global__ __launch_bounds__(NTHREADS, 2) void xeng_cache_kernel(XJob p)
{
    int f, g, w;
    if (!decode_item(p, p.block0 + blockIdx.x, f, g, w)) return;
    process_item_cache<ACC, IN, TILE>(p, f, g, w);
}

// One work item of a batch launch, in the launch's load mode (the narrowest any of its jobs
// needs; a word-load launch still loads whole chunks with single wide loads where a row
// allows it, so jobs with chunk-aligned rows lose nothing, and a single mode keeps one copy
// of the item code in the kernel: two would not fit the register file).
template <int ACC, int IN, int TILE, int MODE>
__device__ __forceinline__ void run_batch_item(const XJob &jb, const XItem &item, uint8_t *lds)
{
    process_item<ACC, IN, TILE, MODE>(jb, item.chan, item.tile, item.window, lds);
}

// Persistent batched kernel: workgroups take (job, channel, tile, window) items off the
// queues until all are empty (see XQueues); every workgroup reaches the exit.
template <int ACC, int IN, int TILE, int MODE>
__global__ __launch_bounds__(NTHREADS, 2) void xeng_mfma_batch_kernel(const XJob *jobs, const XItem *items,
                                                                      XQueues q, unsigned int *counters)
{
    uint8_t *lds = dyn_lds;
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
            // a copy in registers: through a reference every field would be re-read after
            // each store the compiler cannot tell apart from the job table
            const XJob jb = jobs[item.job];
            run_batch_item<ACC, IN, TILE, MODE>(jb, item, lds);
        }
    }
}

// The same over a work list generated on the device (see XGenQueues): the counter of a
// queue numbers its items directly.
template <int ACC, int IN, int TILE, int MODE>
__global__ __launch_bounds__(NTHREADS, 2) void xeng_mfma_batch_gen_kernel(const XJob *jobs, XGenQueues gq,
                                                                          unsigned int *counters)
{
    uint8_t *lds = dyn_lds;
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
            // a copy in registers: through a reference every field would be re-read after
            // each store the compiler cannot tell apart from the job table
            const XJob jb = jobs[item.job];
            run_batch_item<ACC, IN, TILE, MODE>(jb, item, lds);
        }
    }
}

template <int ACC, int IN, int TILE, int MODE>
int launch_mode(const XJob &job, hipStream_t stream)
{
    constexpr int LDS = Tile<ACC, IN, TILE>::LDS_BYTES;
    auto k = xeng_mfma_kernel<ACC, IN, TILE, MODE>;
    if (int e = allow_lds_on_device<xeng_mfma_kernel<ACC, IN, TILE, MODE>>(LDS)) return e;
    hipLaunchKernelGGL(k, dim3((unsigned)job.grid), dim3(NTHREADS), LDS, stream, job);
    return (int)hipGetLastError();
}

template <int ACC, int IN, int TILE>
int launch_one(const XJob &job, hipStream_t stream)
{
    if (job.load_mode == LOAD_VEC) return launch_mode<ACC, IN, TILE, LOAD_VEC>(job, stream);
    if (job.load_mode == LOAD_WORD) return launch_mode<ACC, IN, TILE, LOAD_WORD>(job, stream);
    return launch_mode<ACC, IN, TILE, LOAD_ELEM>(job, stream);
}

template <int ACC, int IN, int TILE, int MODE>
int launch_batch(const XJob *jobs, const XItem *items, const XQueues &q, unsigned int *counters, int nblocks,
                 hipStream_t stream)
{
    constexpr int LDS = Tile<ACC, IN, TILE>::LDS_BYTES;
    auto k = xeng_mfma_batch_kernel<ACC, IN, TILE, MODE>;
    if (int e = allow_lds_on_device<xeng_mfma_batch_kernel<ACC, IN, TILE, MODE>>(LDS)) return e;
    hipLaunchKernelGGL(k, dim3(nblocks), dim3(NTHREADS), LDS, stream, jobs, items, q, counters);
    return (int)hipGetLastError();
}

template <int ACC, int IN, int TILE, int MODE>
int launch_batch_gen(const XJob *jobs, const XGenQueues &g, unsigned int *counters, int nblocks, hipStream_t stream)
{
    constexpr int LDS = Tile<ACC, IN, TILE>::LDS_BYTES;
    auto k = xeng_mfma_batch_gen_kernel<ACC, IN, TILE, MODE>;
    if (int e = allow_lds_on_device<xeng_mfma_batch_gen_kernel<ACC, IN, TILE, MODE>>(LDS)) return e;
    hipLaunchKernelGGL(k, dim3(nblocks), dim3(NTHREADS), LDS, stream, jobs, g, counters);
    return (int)hipGetLastError();
}

template <int ACC, int IN>
int launch_batch_gen_in(const XJob *jobs, const XGenQueues &g, unsigned int *counters, int tile, int mode,
                        int nblocks, hipStream_t stream)
{
    if (tile == 128) {
        if (mode == LOAD_VEC) return launch_batch_gen<ACC, IN, 128, LOAD_VEC>(jobs, g, counters, nblocks, stream);
        if (mode == LOAD_WORD) return launch_batch_gen<ACC, IN, 128, LOAD_WORD>(jobs, g, counters, nblocks, stream);
        return launch_batch_gen<ACC, IN, 128, LOAD_ELEM>(jobs, g, counters, nblocks, stream);
    }
    if (tile == 64) {
        if (mode == LOAD_VEC) return launch_batch_gen<ACC, IN, 64, LOAD_VEC>(jobs, g, counters, nblocks, stream);
        if (mode == LOAD_WORD) return launch_batch_gen<ACC, IN, 64, LOAD_WORD>(jobs, g, counters, nblocks, stream);
        return launch_batch_gen<ACC, IN, 64, LOAD_ELEM>(jobs, g, counters, nblocks, stream);
    }
    return (int)hipErrorInvalidValue;
}

template <int ACC>
int launch_batch_gen_acc(const XJob *jobs, const XGenQueues &g, unsigned int *counters, int in_fmt, int tile,
                         int mode, int nblocks, hipStream_t stream)
{
    if (in_fmt == IN_CI8) return launch_batch_gen_in<ACC, IN_CI8>(jobs, g, counters, tile, mode, nblocks, stream);
    if (in_fmt == IN_CI4) return launch_batch_gen_in<ACC, IN_CI4>(jobs, g, counters, tile, mode, nblocks, stream);
    return (int)hipErrorInvalidValue;
}

template <int ACC, int IN>
int launch_cache_in(const XJob &job, hipStream_t stream)
{
    const dim3 grid((unsigned)job.grid), block(NTHREADS);
    if (job.tile == 128) hipLaunchKernelGGL((xeng_cache_kernel<ACC, IN, 128>), grid, block, 0, stream, job);
    else if (job.tile == 64) hipLaunchKernelGGL((xeng_cache_kernel<ACC, IN, 64>), grid, block, 0, stream, job);
    else return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}

template <int ACC>
int launch_cache_acc(const XJob &job, int in_fmt, hipStream_t stream)
{
    if (in_fmt == IN_CI8) return launch_cache_in<ACC, IN_CI8>(job, stream);
    if (in_fmt == IN_CI4) return launch_cache_in<ACC, IN_CI4>(job, stream);
    return (int)hipErrorInvalidValue;
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

template <int ACC, int IN, int TILE>
int launch_batch_mode(const XJob *jobs, const XItem *items, const XQueues &q, unsigned int *counters, int mode,
                      int nblocks, hipStream_t stream)
{
    if (mode == LOAD_VEC) return launch_batch<ACC, IN, TILE, LOAD_VEC>(jobs, items, q, counters, nblocks, stream);
    if (mode == LOAD_WORD) return launch_batch<ACC, IN, TILE, LOAD_WORD>(jobs, items, q, counters, nblocks, stream);
    return launch_batch<ACC, IN, TILE, LOAD_ELEM>(jobs, items, q, counters, nblocks, stream);
}

template <int ACC, int IN>
int launch_batch_tile(const XJob *jobs, const XItem *items, const XQueues &q, unsigned int *counters, int tile,
                      int mode, int nblocks, hipStream_t stream)
{
    if (tile == 128) return launch_batch_mode<ACC, IN, 128>(jobs, items, q, counters, mode, nblocks, stream);
    if (tile == 64) return launch_batch_mode<ACC, IN, 64>(jobs, items, q, counters, mode, nblocks, stream);
    return (int)hipErrorInvalidValue;
}

template <int ACC>
int launch_batch_in(const XJob *jobs, const XItem *items, const XQueues &q, unsigned int *counters, int in_fmt,
                    int tile, int mode, int nblocks, hipStream_t stream)
{
    if (in_fmt == IN_CI8) return launch_batch_tile<ACC, IN_CI8>(jobs, items, q, counters, tile, mode, nblocks, stream);
    if (in_fmt == IN_CI4) return launch_batch_tile<ACC, IN_CI4>(jobs, items, q, counters, tile, mode, nblocks, stream);
    return (int)hipErrorInvalidValue;
}

}  // namespace
}  // namespace xc

// One arithmetic path's launchers (the kernels of each path are compiled in a translation
// unit of their own, in parallel): plain tiles, cache-staged tiles, batch over a work list,
// batch over a generated work list.
#define XENG_MFMA_PATH(ACC, NAME)                                                                              \
    namespace xc {                                                                                             \
    int launch_mfma_##NAME(const XJob &job, int in_fmt, hipStream_t stream)                                    \
    {                                                                                                          \
        return launch_in<ACC>(job, in_fmt, stream);                                                            \
    }                                                                                                          \
    int launch_mfma_cache_##NAME(const XJob &job, int in_fmt, hipStream_t stream)                              \
    {                                                                                                          \
        return launch_cache_acc<ACC>(job, in_fmt, stream);                                                     \
    }                                                                                                          \
    int launch_mfma_batch_##NAME(const XJob *jobs, const XItem *items, const XQueues &q, unsigned int *counters, \
                                 int in_fmt, int tile, int mode, int nblocks, hipStream_t stream)               \
    {                                                                                                          \
        return launch_batch_in<ACC>(jobs, items, q, counters, in_fmt, tile, mode, nblocks, stream);            \
    }                                                                                                          \
    int launch_mfma_batch_gen_##NAME(const XJob *jobs, const XGenQueues &g, unsigned int *counters, int in_fmt, \
                                     int tile, int mode, int nblocks, hipStream_t stream)                      \
    {                                                                                                          \
        return launch_batch_gen_acc<ACC>(jobs, g, counters, in_fmt, tile, mode, nblocks, stream);              \
    }                                                                                                          \
    }
