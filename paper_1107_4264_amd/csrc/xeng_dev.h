// Device helpers shared by the matrix-core X-engine kernels (gfx950): MFMA wrappers for
// the three operand types, the (re, im) -> (-im, re) pair rotation that turns a real
// product into the imaginary part of a complex one, exact int8 -> fp16 conversion, and
// lane exchange for the epilogue.
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

#include "xeng.h"

namespace xc {
namespace dev {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4v __attribute__((ext_vector_type(4)));

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
    // (re, im) -> (-im, re): swapped halves times (-1, 1), exact
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    const h2 v = __builtin_bit_cast(h2, w);
    const h2 r = __builtin_shufflevector(v, v, 1, 0) * (h2){(_Float16)(-1.0f), (_Float16)1.0f};
    return __builtin_bit_cast(uint32_t, r);
}

template <>
__device__ __forceinline__ uint32_t rotate_pairs<ACC_F8>(uint32_t w)
{
    return __builtin_amdgcn_perm(w, w, 0x02030001u) ^ 0x00800080u;
}

__device__ __forceinline__ int sext4(uint32_t v) { return ((int)(v << 28)) >> 28; }

__device__ __forceinline__ uint32_t f16_bits(int v)
{
    return (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)(short)v);
}

// Two (re, im) int8 pairs packed in one word -> two words of (fp16 re, fp16 im).  For v in
// [-128, 127] the fp16 number with bits 0x6400 | (v ^ 0x80) is exactly 1152 + v, so a byte
// permute and one packed fp16 subtraction convert both parts exactly.
__device__ __forceinline__ void ci8x2_to_f16(uint32_t w, uint32_t &lo, uint32_t &hi)
{
    const uint32_t x = w ^ 0x80808080u;
    const uint32_t a = __builtin_amdgcn_perm(0x64646464u, x, 0x04010400u);
    const uint32_t b = __builtin_amdgcn_perm(0x64646464u, x, 0x04030402u);
    const f16x2 bias = {(_Float16)(-1152.0f), (_Float16)(-1152.0f)};
    lo = __builtin_bit_cast(uint32_t, __builtin_bit_cast(f16x2, a) + bias);
    hi = __builtin_bit_cast(uint32_t, __builtin_bit_cast(f16x2, b) + bias);
}

template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    [&]<int... I>(std::integer_sequence<int, I...>) { (f(std::integral_constant<int, I>{}), ...); }(
        std::make_integer_sequence<int, N>{});
}

// Lanes 2k and 2k+1 exchange values (quad_perm 1,0,3,2).
__device__ __forceinline__ int swap_pair_lanes(int v) { return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false); }

// The value lane l sends in a pair exchange where even lanes send a1 and odd lanes a0, i.e.
// odd ? a0 : a1.  The choice is one bitfield-insert instruction on an all-ones mask of the
// odd lanes, written as (non-volatile) assembly: the compiler must not see it as a choice on
// the lane parity, or it may simplify the operand of the cross-lane move under the parity
// of the receiving lane, which is wrong for the sending one.
__device__ __forceinline__ int odd_lane_mask(int lane) { return -(lane & 1); }
__device__ __forceinline__ int pair_send(int a0, int a1, int odd_mask)
{
    int r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(odd_mask), "v"(a0), "v"(a1));
    return r;
}
__device__ __forceinline__ float pair_send(float a0, float a1, int odd_mask)
{
    return __builtin_bit_cast(float, pair_send(__builtin_bit_cast(int, a0), __builtin_bit_cast(int, a1), odd_mask));
}
__device__ __forceinline__ float swap_pair_lanes(float v)
{
    return __builtin_bit_cast(float, swap_pair_lanes(__builtin_bit_cast(int, v)));
}

}  // namespace dev
}  // namespace xc
