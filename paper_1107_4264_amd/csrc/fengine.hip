// F-engine of the FX correlator (Sec. 2.1) with the corner turn, on gfx950: every input's
// complex 8-bit voltage stream is Fourier transformed F samples at a time (one F-point DFT
// per input and frame, channel k = bin k), scaled by a gain, requantised to 8-bit complex
// samples (each component rounded half away from zero and clipped to [-127, 127]) and
// written in the X-engine's corner-turned order [frame][channel][input] (Sec. 4.1).
//
// One workgroup owns one frame of a group of G inputs; each of its waves transforms one
// input at a time, independently of the others (no workgroup barrier inside a transform).
// The transform is a Stockham autosort FFT of radix-16 passes (and one pass of radix 2, 4
// or 8 when log2 F is not a multiple of 4): a lane gathers its R values of a pass (from the
// input frame in memory for the first pass, from the wave's LDS buffer after that),
// multiplies them by the pass's twiddles (a table of exp(-2 pi i m / F) the workgroup fills
// once), does the R-point DFT in registers, and scatters the results to their sorted
// positions.  A wave issues all its reads of a pass before its writes, so one buffer per
// wave serves in place; the buffer and the tile rows are padded against LDS bank conflicts.  The last pass requantises and drops each channel into an LDS tile
// [channel][G inputs], which leaves as rows of G consecutive inputs per channel: the corner
// turn happens in LDS, and HBM sees each sample once in and once out.

#include <hip/hip_runtime.h>

#include <utility>

#include "xeng.h"

namespace xc {
namespace {

template <int F>
struct FeGeo {
    static constexpr int W = F <= 1024 ? 8 : 4;            // waves per workgroup
    static constexpr int G = F <= 1024 ? 32 : 8;            // inputs per workgroup
    static constexpr int THREADS = 64 * W;
    static constexpr int LOGF = __builtin_ctz(F);
    static constexpr int WAVE_BYTES = 8 * (F + F / 16);     // one transform, complex fp32, padded
    static constexpr int TROW = 2 * G + 16;                 // tile row bytes (padded, 16-byte aligned)
    static constexpr int TW_BYTES = 8 * F;                  // exp(-2 pi i m / F), m < F
    static constexpr int TILE_BYTES = TROW * F;             // requantised [F][G] int8 pairs
    static constexpr int LDS = W * WAVE_BYTES + TW_BYTES + TILE_BYTES;
    static_assert(LDS <= 160 * 1024, "LDS budget");
    static_assert(G % W == 0, "whole rounds");
};

// exp(-2 pi i m / 16): cos and sin of 2 pi m / 16
__device__ __forceinline__ constexpr float c16(int m)
{
    constexpr float c[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f, 0.0f,
                             -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f, -1.0f,
                             -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f, 0.0f,
                             0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
    return c[m & 15];
}
__device__ __forceinline__ constexpr float s16(int m) { return c16(m + 12); }  // sin(x) = cos(x - pi/2)

__device__ __forceinline__ float2 cmul(float2 a, float2 w) { return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x); }

// Calls fn(std::integral_constant<int, i>) for i = 0 .. N-1 (compile-time indices).
template <typename Fn, int... I>
__device__ __forceinline__ void sfor_impl(Fn &&fn, std::integer_sequence<int, I...>)
{
    (fn(std::integral_constant<int, I>{}), ...);
}
template <int N, typename Fn>
__device__ __forceinline__ void sfor(Fn &&fn)
{
    sfor_impl(fn, std::make_integer_sequence<int, N>{});
}

// a * exp(-2 pi i M / 16) for a compile-time M: multiples of pi/2 are exchanges and sign
// changes, odd multiples of pi/4 one shared scale, the rest a complex product.
template <int M>
__device__ __forceinline__ float2 w16(float2 a)
{
    constexpr int m = M & 15;
    constexpr float H = 0.70710678118654752f;
    if constexpr (m == 0) return a;
    else if constexpr (m == 4) return make_float2(a.y, -a.x);
    else if constexpr (m == 8) return make_float2(-a.x, -a.y);
    else if constexpr (m == 12) return make_float2(-a.y, a.x);
    else if constexpr (m == 2) return make_float2(H * (a.x + a.y), H * (a.y - a.x));
    else if constexpr (m == 6) return make_float2(H * (a.y - a.x), -H * (a.x + a.y));
    else if constexpr (m == 10) return make_float2(-H * (a.x + a.y), H * (a.x - a.y));
    else if constexpr (m == 14) return make_float2(H * (a.x - a.y), H * (a.x + a.y));
    else {
        constexpr float c = c16(m), sn = s16(m);
        return make_float2(a.x * c + a.y * sn, a.y * c - a.x * sn);
    }
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// 4-point DFT in place, natural order in and out.
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3)
{
    const float2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = csub(a1, a3);
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = make_float2(t1.x + t3.y, t1.y - t3.x);  // t1 - i t3
    a3 = make_float2(t1.x - t3.y, t1.y + t3.x);  // t1 + i t3
}

// In-register R-point DFT (R = 2, 4, 8, 16), X[k] = sum_n v[n] exp(-2 pi i k n / R), natural
// order in and out: 8 = 2 x 4 and 16 = 4 x 4 (Cooley-Tukey, decimation in time) with the
// twiddles between the stages at compile time.
template <int R>
__device__ __forceinline__ void dft_small(float2 (&v)[R])
{
    if constexpr (R == 2) {
        const float2 t = v[0];
        v[0] = cadd(t, v[1]);
        v[1] = csub(t, v[1]);
    } else if constexpr (R == 4) {
        dft4(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 8) {
        float2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        dft4(e[0], e[1], e[2], e[3]);
        dft4(o[0], o[1], o[2], o[3]);
        sfor<4>([&](auto K) __attribute__((always_inline)) {
            constexpr int k = decltype(K)::value;
            const float2 t = w16<2 * k>(o[k]);  // exp(-2 pi i k / 8)
            v[k] = cadd(e[k], t);
            v[k + 4] = csub(e[k], t);
        });
    } else {
        static_assert(R == 16, "radix 2, 4, 8 or 16");
        // n = 4 n1 + n2, k = k1 + 4 k2: 4-point DFTs over n1, twiddles exp(-2 pi i n2 k1 / 16),
        // 4-point DFTs over n2
        float2 y[4][4];
        sfor<4>([&](auto N2) __attribute__((always_inline)) {
            constexpr int n2 = decltype(N2)::value;
            y[n2][0] = v[n2];
            y[n2][1] = v[4 + n2];
            y[n2][2] = v[8 + n2];
            y[n2][3] = v[12 + n2];
            dft4(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
            sfor<4>([&](auto K1) __attribute__((always_inline)) {
                constexpr int k1 = decltype(K1)::value;
                y[n2][k1] = w16<n2 * k1>(y[n2][k1]);
            });
        });
        sfor<4>([&](auto K1) __attribute__((always_inline)) {
            constexpr int k1 = decltype(K1)::value;
            float2 b0 = y[0][k1], b1 = y[1][k1], b2 = y[2][k1], b3 = y[3][k1];
            dft4(b0, b1, b2, b3);
            v[k1] = b0;
            v[k1 + 4] = b1;
            v[k1 + 8] = b2;
            v[k1 + 12] = b3;
        });
    }
}

__device__ __forceinline__ int requant(float v)
{
    const float r = roundf(v);  // halves away from zero
    return (int)fminf(fmaxf(r, -127.0f), 127.0f);
}

extern __shared__ __attribute__((aligned(16))) uint8_t fe_lds[];

// First-pass inputs of one transform, loaded ahead (the first pass has radix 16: values
// x[j + 16... ] of j = lane + 64 q).
template <int F>
struct FeFirst {
    static constexpr int JPL = (F / 16 + 63) / 64;
    uint32_t v[JPL][16];
};

template <int F>
__device__ __forceinline__ void load_first(FeFirst<F> &fx, const uint16_t *src, int lane)
{
    constexpr int JC = F / 16;
#pragma unroll
    for (int q = 0; q < FeFirst<F>::JPL; ++q) {
        const int j = lane + 64 * q;
        if (JC % 64 != 0 && j >= JC) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) fx.v[q][r] = src[j + r * JC];
    }
}

// Position of point k in a wave's buffer: one float2 of padding after every 16, so that the
// first pass's stores (16 consecutive points per lane) and the tile-row stores spread over
// the LDS banks.
__device__ __forceinline__ int pad(int k) { return k + (k >> 4); }

struct FeArgs {
    float2 *buf;          // this wave's LDS buffer
    const float2 *tw;     // twiddle table
    int8_t *tile;         // requantised tile [F][G]
    float2 *spec;         // spectra output of this input and frame (stride nin), or null
    int64_t spec_stride;
    int g, lane;
    float gain;
};

// One Stockham pass of radix R over a transform of F points, after NS points of output
// sorted so far.  j = 0 .. F/R - 1: gather x[j + r F/R], twiddle by exp(-2 pi i (j mod NS)
// r / (NS R)), R-point DFT, scatter to (j / NS) NS R + (j mod NS) + r NS.
template <int F, int G, int R, int NS, bool LAST, bool SPECTRA>
__device__ __forceinline__ void fft_pass(const FeArgs &a, const FeFirst<F> &fx)
{
    constexpr int JC = F / R, JPL = (JC + 63) / 64;
    constexpr int TROW = 2 * G + 16;
    float2 v[JPL][R];
#pragma unroll
    for (int q = 0; q < JPL; ++q) {
        const int j = a.lane + 64 * q;
        if (JC % 64 != 0 && j >= JC) continue;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if constexpr (NS == 1) {
                const uint32_t w = fx.v[q][r];
                v[q][r] = make_float2((float)(int8_t)(w & 0xFF), (float)(int8_t)(w >> 8));
            } else {
                v[q][r] = a.buf[pad(j + r * JC)];
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < JPL; ++q) {
        const int j = a.lane + 64 * q;
        if (JC % 64 != 0 && j >= JC) continue;
        const int jm = NS == 1 ? 0 : (j & (NS - 1));
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], a.tw[(jm * r * (F / (NS * R))) & (F - 1)]);
        }
        dft_small<R>(v[q]);
        const int d0 = (j / NS) * NS * R + jm;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int k = d0 + r * NS;
            if constexpr (!LAST) {
                a.buf[pad(k)] = v[q][r];
            } else if constexpr (SPECTRA) {
                a.spec[(int64_t)k * a.spec_stride] = make_float2(a.gain * v[q][r].x, a.gain * v[q][r].y);
            } else {
                const uint32_t p =
                    (uint32_t)(requant(a.gain * v[q][r].x) & 0xFF) | ((uint32_t)(requant(a.gain * v[q][r].y) & 0xFF) << 8);
                *(uint16_t *)(a.tile + k * TROW + 2 * a.g) = (uint16_t)p;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// The passes of an F-point transform: radix 16 while at least four bits remain, then one
// pass of radix 2^REM.
template <int F, int G, int NS, int REM, bool SPECTRA>
__device__ __forceinline__ void fft_passes(const FeArgs &a, const FeFirst<F> &fx)
{
    constexpr int LR = REM >= 4 ? 4 : REM;
    constexpr bool LAST = REM <= 4;
    static_assert(NS > 1 || LR == 4, "the first pass has radix 16");
    fft_pass<F, G, (1 << LR), NS, LAST, SPECTRA>(a, fx);
    if constexpr (!LAST) fft_passes<F, G, NS * (1 << LR), REM - LR, SPECTRA>(a, fx);
}

// SPECTRA: write the scaled spectra as complex fp32 [frame][channel][input] instead of the
// requantised samples (no tile; for checking the transform itself).
template <int F, bool SPECTRA>
__global__ __launch_bounds__(FeGeo<F>::THREADS) void fengine_kernel(const int8_t *__restrict__ in, void *__restrict__ out,
                                                                    int nin, int64_t nsamp, int nframes, float gain)
{
    using Ge = FeGeo<F>;
    constexpr int G = Ge::G, W = Ge::W;
    const int ngroups = (nin + G - 1) / G;
    const int t = (int)(blockIdx.x / ngroups);
    const int i0 = (int)(blockIdx.x % ngroups) * G;
    if (t >= nframes) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float2 *tw = (float2 *)(fe_lds + W * Ge::WAVE_BYTES);
    int8_t *tile = (int8_t *)(fe_lds + W * Ge::WAVE_BYTES + Ge::TW_BYTES);

    // twiddles exp(-2 pi i m / F) (sincospi of an exact multiple of 2/F)
    for (int m = threadIdx.x; m < F; m += Ge::THREADS) {
        float s, c;
        sincospif(-2.0f * (float)m / (float)F, &s, &c);
        tw[m] = make_float2(c, s);
    }
    __syncthreads();

    const int nin_here = min(G, nin - i0);
    FeArgs a;
    a.buf = (float2 *)(fe_lds + wave * Ge::WAVE_BYTES);
    a.tw = tw;
    a.tile = tile;
    a.lane = lane;
    a.gain = gain;
    a.spec_stride = nin;
    // the next input's frame is loaded while the current one is transformed
    auto frame = [&](int g) { return (const uint16_t *)in + ((int64_t)(i0 + g) * nsamp + (int64_t)t * F); };
    auto transform = [&](int g, const FeFirst<F> &fx) __attribute__((always_inline)) {
        a.g = g;
        a.spec = SPECTRA ? (float2 *)out + ((int64_t)t * F * nin + i0 + g) : nullptr;
        fft_passes<F, G, 1, Ge::LOGF, SPECTRA>(a, fx);
    };
    FeFirst<F> fx0, fx1;  // two named buffers (an indexed pair would live in scratch memory)
    if (wave < nin_here) load_first<F>(fx0, frame(wave), lane);
    for (int g = wave; g < nin_here; g += 2 * W) {
        if (g + W < nin_here) load_first<F>(fx1, frame(g + W), lane);
        transform(g, fx0);
        if (g + W >= nin_here) break;
        if (g + 2 * W < nin_here) load_first<F>(fx0, frame(g + 2 * W), lane);
        transform(g + W, fx1);
    }
    if constexpr (!SPECTRA) {
        __syncthreads();
        // tile rows -> out[t][k][i0 .. i0 + nin_here)
        int8_t *o = (int8_t *)out + 2 * ((int64_t)t * F * nin + i0);
        if (nin_here == G && nin % 8 == 0 && ((uintptr_t)out & 15) == 0) {
            constexpr int PIECES = G / 8;  // 16 bytes = 8 inputs
            for (int e = threadIdx.x; e < F * PIECES; e += Ge::THREADS) {
                const int k = e / PIECES, pc = e - k * PIECES;
                *(uint4 *)(o + 2 * ((int64_t)k * nin + 8 * pc)) = *(const uint4 *)(tile + k * Ge::TROW + 16 * pc);
            }
        } else {
            for (int e = threadIdx.x; e < F * G; e += Ge::THREADS) {
                const int k = e / G, g = e - k * G;
                if (g < nin_here) *(uint16_t *)(o + 2 * ((int64_t)k * nin + g)) = *(const uint16_t *)(tile + k * Ge::TROW + 2 * g);
            }
        }
    }
}

template <int F, bool SPECTRA>
int launch_f(const int8_t *in, void *out, int nin, int64_t nsamp, int nframes, float gain, hipStream_t stream)
{
    constexpr int LDS = FeGeo<F>::LDS;
    if (int e = allow_lds_on_device<fengine_kernel<F, SPECTRA>>(LDS)) return e;
    const int64_t ngroups = (nin + FeGeo<F>::G - 1) / FeGeo<F>::G;
    const int64_t blocks = ngroups * nframes;
    if (blocks <= 0) return 0;
    if (blocks > 0x7FFFFFFF) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL((fengine_kernel<F, SPECTRA>), dim3((unsigned)blocks), dim3(FeGeo<F>::THREADS), LDS, stream, in,
                       out, nin, nsamp, nframes, gain);
    return (int)hipGetLastError();
}

template <bool SPECTRA>
int launch_fengine_t(const int8_t *in, void *out, int nin, int nchan, int64_t nsamp, int nframes, float gain,
                     hipStream_t stream)
{
    switch (nchan) {
    case 64: return launch_f<64, SPECTRA>(in, out, nin, nsamp, nframes, gain, stream);
    case 128: return launch_f<128, SPECTRA>(in, out, nin, nsamp, nframes, gain, stream);
    case 256: return launch_f<256, SPECTRA>(in, out, nin, nsamp, nframes, gain, stream);
    case 512: return launch_f<512, SPECTRA>(in, out, nin, nsamp, nframes, gain, stream);
    case 1024: return launch_f<1024, SPECTRA>(in, out, nin, nsamp, nframes, gain, stream);
    case 2048: return launch_f<2048, SPECTRA>(in, out, nin, nsamp, nframes, gain, stream);
    default: return (int)hipErrorInvalidValue;
    }
}

}  // namespace

int launch_fengine(const void *in, void *out, int nin, int nchan, int64_t nsamp, int nframes, float gain,
                   bool spectra, hipStream_t stream)
{
    const int8_t *p = (const int8_t *)in;
    return spectra ? launch_fengine_t<true>(p, out, nin, nchan, nsamp, nframes, gain, stream)
                   : launch_fengine_t<false>(p, out, nin, nchan, nsamp, nframes, gain, stream);
}

}  // namespace xc
