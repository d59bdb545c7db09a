// F-engine of the FX correlator (Sec. 2.1) with the corner turn, on gfx950: every input's
// complex 8-bit voltage stream is Fourier transformed F samples at a time (one F-point DFT
// per input and frame, channel k = bin k), scaled by a gain, requantised to 8-bit complex
// samples (each component rounded half away from zero and clipped to [-127, 127]) and
// written in the X-engine's corner-turned order [frame][channel][input] (Sec. 4.1).
//
// One workgroup owns one frame of a group of G inputs.  Its four waves transform one input
// each at a time, in LDS (radix-2 decimation in time: samples stored at their bit-reversed
// index as they arrive, then log2 F passes of butterflies with twiddles from a table the
// workgroup fills once), and drop the requantised channels into an LDS tile [channel][G
// inputs]; the tile leaves as rows of G consecutive inputs per channel, so the corner turn
// costs no extra pass over HBM.  Reads are the inputs' contiguous frames.

#include <hip/hip_runtime.h>

#include "xeng.h"

namespace xc {
namespace {

constexpr int FE_THREADS = 256;  // four waves

// Inputs per workgroup for an F-point transform: 32 (64-byte rows of the output tile) up
// to F = 1024, fewer above so the tile stays at 64 KiB.
template <int F>
struct FeGeo {
    static constexpr int G = F <= 1024 ? 32 : 32768 / F;
    static constexpr int LOGF = __builtin_ctz(F);
    static constexpr int WAVE_BYTES = 8 * F;               // one transform, complex fp32
    static constexpr int TW_BYTES = 4 * F;                 // F/2 twiddles
    static constexpr int TILE_BYTES = 2 * F * G;           // requantised [F][G] int8 pairs
    static constexpr int LDS = 4 * WAVE_BYTES + TW_BYTES + TILE_BYTES;
    static_assert(LDS <= 160 * 1024, "LDS budget");
};

__device__ __forceinline__ int bitrev(int n, int bits) { return (int)(__builtin_bitreverse32((uint32_t)n) >> (32 - bits)); }

__device__ __forceinline__ int requant(float v)
{
    const float r = roundf(v);  // halves away from zero
    return (int)fminf(fmaxf(r, -127.0f), 127.0f);
}

extern __shared__ __attribute__((aligned(16))) uint8_t fe_lds[];

// SPECTRA: write the scaled spectra as complex fp32 [frame][channel][input] instead of the
// requantised samples (no tile; for checking the transform itself).
template <int F, bool SPECTRA>
__global__ __launch_bounds__(FE_THREADS) void fengine_kernel(const int8_t *__restrict__ in, void *__restrict__ out,
                                                             int nin, int64_t nsamp, int nframes, float gain)
{
    using Ge = FeGeo<F>;
    constexpr int G = Ge::G;
    const int ngroups = (nin + G - 1) / G;
    const int t = (int)(blockIdx.x / ngroups);
    const int i0 = (int)(blockIdx.x % ngroups) * G;
    if (t >= nframes) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float2 *tw = (float2 *)(fe_lds + 4 * Ge::WAVE_BYTES);
    float2 *buf = (float2 *)(fe_lds + wave * Ge::WAVE_BYTES);
    int8_t *tile = (int8_t *)(fe_lds + 4 * Ge::WAVE_BYTES + Ge::TW_BYTES);

    // twiddles exp(-2 pi i k / F), k < F/2 (sincospi of an exact multiple of 2/F)
    for (int k = threadIdx.x; k < F / 2; k += FE_THREADS) {
        float s, c;
        sincospif(-2.0f * (float)k / (float)F, &s, &c);
        tw[k] = make_float2(c, s);
    }
    __syncthreads();

    const int nin_here = min(G, nin - i0);
    // every wave runs the same number of rounds (barriers inside the transform)
    for (int r = 0; r < (G + 3) / 4; ++r) {
        const int g = 4 * r + wave;
        const bool have = g < nin_here;
        if (have) {
            // frame t of input i0 + g: F samples, two per lane and load
            const int16_t *src = (const int16_t *)in + ((int64_t)(i0 + g) * nsamp + (int64_t)t * F);
            for (int n = 2 * lane; n < F; n += 128) {
                const uint32_t w = *(const uint32_t *)(src + n);
                const float r0 = (float)(int8_t)(w & 0xFF), m0 = (float)(int8_t)((w >> 8) & 0xFF);
                const float r1 = (float)(int8_t)((w >> 16) & 0xFF), m1 = (float)(int8_t)(w >> 24);
                buf[bitrev(n, Ge::LOGF)] = make_float2(r0, m0);
                buf[bitrev(n + 1, Ge::LOGF)] = make_float2(r1, m1);
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int s = 0; s < Ge::LOGF; ++s) {
            const int half = 1 << s;
            if (have) {
                for (int b = lane; b < F / 2; b += 64) {
                    const int pos = b & (half - 1);
                    const int i = ((b >> s) << (s + 1)) + pos, j = i + half;
                    const float2 w = tw[pos << (Ge::LOGF - 1 - s)];
                    const float2 u = buf[i], v = buf[j];
                    const float2 vw = make_float2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
                    buf[i] = make_float2(u.x + vw.x, u.y + vw.y);
                    buf[j] = make_float2(u.x - vw.x, u.y - vw.y);
                }
            }
            __syncthreads();
        }
        if (have) {
            if constexpr (SPECTRA) {
                float2 *o = (float2 *)out;
                for (int k = lane; k < F; k += 64) {
                    const float2 v = buf[k];
                    o[((int64_t)t * F + k) * nin + i0 + g] = make_float2(gain * v.x, gain * v.y);
                }
            } else {
                for (int k = lane; k < F; k += 64) {
                    const float2 v = buf[k];
                    const uint32_t q = (uint32_t)(requant(gain * v.x) & 0xFF) | ((uint32_t)(requant(gain * v.y) & 0xFF) << 8);
                    *(uint16_t *)(tile + 2 * (k * G + g)) = (uint16_t)q;
                }
            }
        }
        __syncthreads();
    }
    if constexpr (!SPECTRA) {
        // tile rows -> out[t][k][i0 .. i0 + nin_here): 4-byte pieces (two inputs)
        int8_t *o = (int8_t *)out;
        constexpr int PIECES = G / 2;
        for (int e = threadIdx.x; e < F * PIECES; e += FE_THREADS) {
            const int k = e / PIECES, pc = e - k * PIECES;
            const int g = 2 * pc;
            int8_t *dst = o + 2 * (((int64_t)t * F + k) * nin + i0 + g);
            const uint32_t v = *(const uint32_t *)(tile + 2 * (k * G + g));
            if (g + 1 < nin_here) {
                if ((((uintptr_t)dst) & 3) == 0) {
                    *(uint32_t *)dst = v;
                } else {
                    *(uint16_t *)dst = (uint16_t)v;
                    *(uint16_t *)(dst + 2) = (uint16_t)(v >> 16);
                }
            } else if (g < nin_here) {
                *(uint16_t *)dst = (uint16_t)v;
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
    hipLaunchKernelGGL((fengine_kernel<F, SPECTRA>), dim3((unsigned)blocks), dim3(FE_THREADS), LDS, stream, in, out,
                       nin, nsamp, nframes, gain);
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
