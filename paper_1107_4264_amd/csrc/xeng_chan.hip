// Whole-channel X-engine on the CDNA4 matrix cores (gfx950) for arrays of up to 256
// complex 8-bit inputs.
//
// For such arrays one workgroup owns all the baselines of a channel (the whole lower
// triangle of Eq. 4 at 32x32 block granularity: 8 block rows, 36 blocks), so every input
// sample is read from HBM exactly once, as whole 512-byte rows of the [time][channel]
// [input] layout of Sec. 4.1; splitting a row between tiles costs half the bandwidth on
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

#include "xeng_chan_dev.h"

namespace xc {
namespace {

template <int ACC, int W, int V>
__device__ __forceinline__ void run_wave(const XJob &p, int lane)
{
    using O = COp<ACC>;
    using G = Geom<ACC, V>;
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
        // raw ring with transposing reads.  By default only the waves with five blocks (0..3)
        // convert: the four-block waves share their SIMDs with them and are the ones the
        // barriers wait for; variant bit 2 spreads the conversion over all eight waves.
        // Instruction u of converting wave W covers the 16-input group ig = 4 (u % 4) +
        // lane / 16 at sample group q = (UPW / 4) W + u / 4; units u and u + 4 differ by four
        // sample rows.
        constexpr int CW = (V & 4) ? 8 : 4;            // converting waves
        constexpr int UPW = 16 * G::QUADS / 4 / CW;    // conversion instructions per converting wave
        constexpr int UPK = UPW / NKS;                 // of them per K-step
        static_assert(UPK * NKS == UPW && UPK >= 1 && UPK <= 2, "whole conversion units per K-step");
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
                    s16x4 cv[UPK];
                    if constexpr (W < CW) {
#pragma unroll
                        for (int j = 0; j < UPK; ++j) cv[j] = convert_read(UPK * k + j, csrc);
                    }
                    if constexpr (k + 1 < NKS) read_staged<S, k + 1>(lvf, nxt);
                    __builtin_amdgcn_sched_barrier(0);
                    mma_step<ACC, S>(cur, acc, [&]() __attribute__((always_inline)) { copy_at(K, rs, dst); },
                                     [&]() __attribute__((always_inline)) {
                                         if constexpr (W < CW) {
#pragma unroll
                                             for (int j = 0; j < UPK; ++j) convert_write(UPK * k + j, cv[j], cdst);
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

// Variant V: bit 0 one ring slot fewer (Geom), bit 1 the other assignment of the work lists
// to the older and younger wave of each SIMD, bit 2 (fp16) the conversion on all eight waves.
template <int ACC, int V>
__global__ __launch_bounds__(CT, 1) void xeng_chan_kernel(XJob p)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // Waves w and w + 4 share a SIMD and the older one (w) wins its issue conflicts.  By
    // default the fp16 path gives it the five-block list and the conversion; the int8 path
    // runs faster with the four-block squares on the older waves.
    constexpr int X = (ACC == ACC_I8 ? 4 : 0) ^ ((V & 2) ? 4 : 0);
    switch (wave) {
    case 0: run_wave<ACC, 0 ^ X, V>(p, lane); break;
    case 1: run_wave<ACC, 1 ^ X, V>(p, lane); break;
    case 2: run_wave<ACC, 2 ^ X, V>(p, lane); break;
    case 3: run_wave<ACC, 3 ^ X, V>(p, lane); break;
    case 4: run_wave<ACC, 4 ^ X, V>(p, lane); break;
    case 5: run_wave<ACC, 5 ^ X, V>(p, lane); break;
    case 6: run_wave<ACC, 6 ^ X, V>(p, lane); break;
    default: run_wave<ACC, 7 ^ X, V>(p, lane); break;
    }
}


template <int ACC, int V>
int launch_chan_var(const XJob &job, hipStream_t stream)
{
    constexpr int LDS = Geom<ACC, V>::LDS;
    if (int e = allow_lds_on_device<xeng_chan_kernel<ACC, V>>(LDS)) return e;
    hipLaunchKernelGGL((xeng_chan_kernel<ACC, V>), dim3((unsigned)job.grid), dim3(CT), LDS, stream, job);
    return (int)hipGetLastError();
}

template <int ACC>
int launch_chan_acc(const XJob &job, hipStream_t stream)
{
    switch (job.variant) {
    case 0: return launch_chan_var<ACC, 0>(job, stream);
    case 1: return launch_chan_var<ACC, 1>(job, stream);
    case 2: return launch_chan_var<ACC, 2>(job, stream);
    case 3: return launch_chan_var<ACC, 3>(job, stream);
    default: break;
    }
    if constexpr (ACC == ACC_F16) {
        switch (job.variant) {
        case 4: return launch_chan_var<ACC, 4>(job, stream);
        case 5: return launch_chan_var<ACC, 5>(job, stream);
        case 6: return launch_chan_var<ACC, 6>(job, stream);
        case 7: return launch_chan_var<ACC, 7>(job, stream);
        default: break;
        }
    }
    return (int)hipErrorInvalidValue;
}

}  // namespace

int launch_chan(const XJob &job, int acc, hipStream_t stream)
{
    if (job.grid <= 0) return 0;
    if (acc == ACC_I8) return launch_chan_acc<ACC_I8>(job, stream);
    if (acc == ACC_F16) return launch_chan_acc<ACC_F16>(job, stream);
    return (int)hipErrorInvalidValue;
}

}  // namespace xc
