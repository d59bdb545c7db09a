// Host-side planner (no GPU calls).
#include "plan.h"

#include <limits.h>

#include "xcorr.h"
#include "xeng.h"

namespace xc {

size_t in_sample_bytes(int in_fmt)
{
    switch (in_fmt) {
    case IN_CI8: return 2;
    case IN_CI4: return 1;
    case IN_CF32: return 8;
    default: return 0;
    }
}

size_t out_value_bytes(int out_dtype)
{
    switch (out_dtype) {
    case OUT_CI32: return 8;
    case OUT_CI64: return 16;
    case OUT_C64: return 8;
    case OUT_C128: return 16;
    default: return 0;
    }
}

int default_max_abs(int in_fmt, int acc)
{
    if (in_fmt == IN_CI4) return 8;
    if (in_fmt == IN_CI8) return acc == ACC_I8 ? 127 : 128;
    return 0;
}

static int max_abs_cap(int in_fmt, int acc)
{
    if (in_fmt == IN_CI4) return 8;
    if (in_fmt == IN_CI8) return acc == ACC_I8 ? 127 : 128;
    return 0;
}

// One sample adds at most |ar*br| + |ai*bi| <= 2*m^2 to a real or imaginary sum.
int64_t window_limit(int in_fmt, int acc, int max_abs)
{
    if (in_fmt < IN_CI8 || in_fmt > IN_CF32 || acc < ACC_F32_CMAC || acc > ACC_LAST) return -1;
    if (in_fmt == IN_CF32) return acc == ACC_F32_CMAC ? INT64_MAX : -1;
    if (max_abs < 1 || max_abs > max_abs_cap(in_fmt, acc)) return -1;
    const int64_t per = 2 * (int64_t)max_abs * max_abs;
    if (acc == ACC_I8) return ((int64_t)INT32_MAX) / per;
    return ((int64_t)1 << 24) / per;  // every fp32 partial sum of integers <= 2^24 is exact
}

void tile_coords(int64_t g, int64_t *bx, int64_t *by)
{
    // b = floor((isqrt(8g + 1) - 1) / 2), with isqrt by Newton iteration on integers.
    const uint64_t n = 8 * (uint64_t)g + 1;
    uint64_t x = n, y = (x + 1) / 2;
    while (y < x) {
        x = y;
        y = (x + n / x) / 2;
    }
    int64_t b = (int64_t)((x - 1) / 2);
    while (b * (b + 1) / 2 > g) --b;
    while ((b + 1) * (b + 2) / 2 <= g) ++b;
    *by = b;
    *bx = g - b * (b + 1) / 2;
}

bool chan_kernel_ok(int nin, int in_fmt, int acc)
{
    return in_fmt == IN_CI8 && (acc == ACC_I8 || acc == ACC_F16) && nin % 8 == 0 && nin >= 1 && nin <= CHAN_TILE;
}

bool super_kernel_ok(int nin, int nchan, int64_t window, int in_fmt, int acc, int max_abs)
{
    const bool fmt_ok = (in_fmt == IN_CI4 && (acc == ACC_I8 || acc == ACC_F8 || acc == ACC_F6)) ||
                        (in_fmt == IN_CI8 && acc == ACC_I8);
    if (!fmt_ok || nin % 16 != 0 || nin <= 256 || nin > 2048) return false;
    // the copy offsets of a block (32 rows) stay below 2^32 bytes
    if (32 * (int64_t)nchan * nin * (int64_t)in_sample_bytes(in_fmt) >= ((int64_t)1 << 32)) return false;
    // fp8 operands and int8 operands from 8-bit samples are the samples themselves (the
    // usual windows); int8 operands from 4-bit samples are 8 x the samples (16 x on the
    // rectangles' row side), so every window must stay within the int32 limit of the
    // scaled sums, at most 2 (16 m) (8 m) per sample
    if (acc == ACC_F8 || in_fmt == IN_CI8) return true;
    if (acc == ACC_F6) return true;  // (its windows: see make_plan)
    const int64_t m = max_abs;
    return m >= 1 && window <= (int64_t)2147483647 / (256 * m * m);
}

int64_t computed_pairs_per_sample(int nin, int tile, int acc)
{
    // whole-channel kernel: all 36 blocks of the 8x8-block triangle, whatever nin
    if (tile == CHAN_TILE) return 36 * 32 * 32;
    // super-tiles: S triangles of 36 blocks and S (S - 1) rectangles of 32 blocks
    if (tile == SUPER_TILE) {
        const int64_t s = (nin + 255) / 256;
        return (s * 36 + s * (s - 1) * 32) * 32 * 32;
    }
    const int64_t nts = (nin + tile - 1) / tile;
    if (acc == ACC_F32_CMAC) return nts * (nts + 1) / 2 * (int64_t)tile * tile;
    // MFMA kernels: 32x32 blocks, skipping blocks strictly above the diagonal of a diagonal
    // tile and blocks that start beyond the last input.
    const int nbs = tile / 32;
    int64_t total = 0;
    for (int64_t by = 0; by < nts; ++by)
        for (int64_t bx = 0; bx <= by; ++bx)
            for (int r = 0; r < nbs; ++r)
                for (int c = 0; c < nbs; ++c) {
                    if (bx == by && r < c) continue;
                    if (by * tile + r * 32 >= nin || bx * tile + c * 32 >= nin) continue;
                    total += 32 * 32;
                }
    return total;
}

int kernel_variants(int tile, int acc)
{
    if (acc == ACC_F32_CMAC) return 1;
    if (tile == CHAN_TILE) return acc == ACC_F16 ? 8 : 4;
    if (tile == SUPER_TILE) return acc == ACC_F6 ? 2 : 4;
    return 1;
}

int make_plan(int nstation, int npol, int nchan, int ntime, int in_fmt, int acc, int max_abs,
              int tile_override, Plan *pl, std::string *err, int window_req, int staging, int variant)
{
    if (!pl) {
        *err = "null plan";
        return XCORR_ERR_INVALID_ARG;
    }
    if (nstation < 1 || (npol != 1 && npol != 2) || nchan < 1 || ntime < 0) {
        *err = "need nstation >= 1, npol in {1, 2}, nchan >= 1, ntime >= 0";
        return XCORR_ERR_INVALID_ARG;
    }
    if (in_fmt < IN_CI8 || in_fmt > IN_CF32 || acc < ACC_F32_CMAC || acc > ACC_LAST) {
        *err = "unknown input format or arithmetic path";
        return XCORR_ERR_INVALID_ARG;
    }
    if (in_fmt == IN_CF32 && acc != ACC_F32_CMAC) {
        *err = "float input is only accepted by the FP32 CMAC path";
        return XCORR_ERR_UNSUPPORTED;
    }
    if (window_req < 0) {
        *err = "window must be >= 0 (0: the longest exact window)";
        return XCORR_ERR_INVALID_ARG;
    }
    if (staging != 0 && staging != 1) {
        *err = "staging must be 0 (LDS) or 1 (caches)";
        return XCORR_ERR_INVALID_ARG;
    }
    if (staging == 1 && acc == ACC_F32_CMAC) {
        *err = "the FP32 CMAC kernel always stages its operands in LDS";
        return XCORR_ERR_UNSUPPORTED;
    }
    const int64_t nin64 = (int64_t)nstation * npol;
    if (nin64 > 65536) {
        *err = "at most 65536 inputs (stations x polarisations)";
        return XCORR_ERR_RANGE;
    }
    if (max_abs == 0) max_abs = default_max_abs(in_fmt, acc);
    if (in_fmt != IN_CF32 && (max_abs < 1 || max_abs > max_abs_cap(in_fmt, acc))) {
        *err = "max_abs out of range for the sample format";
        return XCORR_ERR_INVALID_ARG;
    }
    if (acc == ACC_F8 && max_abs > 16) {
        *err = "fp8 e4m3 is exact only for |sample| <= 16: use CI4 or declare max_abs <= 16";
        return XCORR_ERR_UNSUPPORTED;
    }
    if (acc == ACC_F6 && max_abs > 8) {
        *err = "fp6 e3m2 is exact only for |sample| <= 8: use CI4 or declare max_abs <= 8";
        return XCORR_ERR_UNSUPPORTED;
    }
    Plan p;
    p.nstation = nstation;
    p.npol = npol;
    p.nchan = nchan;
    p.ntime = ntime;
    p.in_fmt = in_fmt;
    p.acc = acc;
    p.max_abs = in_fmt == IN_CF32 ? 0 : max_abs;
    p.window_req = window_req;
    p.staging = staging;
    p.nin = (int)nin64;

    // Accumulation windows (Sec. 2.3: accumulators wider than the data): the longest exact
    // window, rounded down to whole 64-sample blocks, or the caller's shorter one.
    const int64_t lim = window_limit(in_fmt, acc, in_fmt == IN_CF32 ? 1 : max_abs);
    if (window_req > 0 && window_req > lim) {
        *err = "window longer than the exact limit of the accumulators (see xcorr_window_limit)";
        return XCORR_ERR_UNSUPPORTED;
    }
    const int64_t wmax = window_req > 0 ? window_req : lim;
    if (ntime <= wmax) {
        p.window = ntime > 0 ? ntime : 1;
        p.nwindows = ntime > 0 ? 1 : 0;
    } else {
        const int64_t w = window_req > 0 ? window_req : (lim >= 64 ? (lim / 64) * 64 : lim);
        p.window = (int)w;
        p.nwindows = (int)((ntime + w - 1) / w);
    }

    int tile = acc == ACC_F32_CMAC ? 64 : (p.nin > 64 ? 128 : 64);
    // Above 192 inputs the whole-channel kernel computes at most 36/28 of the useful blocks
    // and reads every sample once, in whole rows.
    if (chan_kernel_ok(p.nin, in_fmt, acc) && p.nin > 192 && !staging) tile = CHAN_TILE;
    // Above 256 inputs of 4-bit samples on the int8 / fp8 / fp6 paths and of 8-bit samples on
    // the int8 path, super-tiles (whole 256-input pieces per workgroup, operands widened or
    // moved once per block in LDS, or on the fp6 path made once by a pre-pass) when their
    // padding of the last super-row costs at most 15 % more computed blocks than 128-tiles
    // (equal at multiples of 256; the pieces run 1.15-1.3x faster per block, the fp6 ones
    // 3.5x).
    // fp6 super-tiles: the pre-pass's units hold whole blocks of 32 samples, so every window
    // must start on one
    const bool super_ok = super_kernel_ok(p.nin, nchan, p.window, in_fmt, acc, max_abs) &&
                          (acc != ACC_F6 || p.nwindows <= 1 || p.window % 32 == 0);
    if (!staging && super_ok &&
        computed_pairs_per_sample(p.nin, SUPER_TILE, acc) * 100 <= computed_pairs_per_sample(p.nin, 128, acc) * 115)
        tile = SUPER_TILE;
    if (tile_override) {
        bool ok;
        if (acc == ACC_F32_CMAC) ok = tile_override == 64;
        else if (tile_override == CHAN_TILE) ok = !staging && chan_kernel_ok(p.nin, in_fmt, acc);
        else if (tile_override == SUPER_TILE)
            ok = !staging && super_ok;
        else ok = tile_override == 64 || tile_override == 128;
        if (!ok) {
            *err = staging && (tile_override == CHAN_TILE || tile_override == SUPER_TILE)
                       ? "staging through the caches runs the tiled kernel: tile 64 or 128"
                   : tile_override == CHAN_TILE
                       ? "tile 256 (whole channel) needs CI8 input, the int8 or fp16 path and nin <= 256, a multiple of 8"
                   : tile_override == SUPER_TILE
                       ? "tile 512 (super-tiles) needs CI4 input on the int8, fp8 or fp6 path or CI8 input on the "
                         "int8 path, nin a multiple of 16 in 272..2048, for CI4 on the int8 path windows of at most "
                         "(2^31-1) / (256 max_abs^2) samples, on the fp6 path windows of whole 32-sample blocks"
                       : "unsupported tile size";
            return XCORR_ERR_INVALID_ARG;
        }
        tile = tile_override;
    }
    p.tile = tile;
    if (variant < 0 || variant >= kernel_variants(tile, acc)) {
        *err = "kernel variant out of range for the kernel shape (whole channel 0..3, fp16 0..7, super-tiles 0..3, fp6 "
                "super-tiles 0..1, others 0)";
        return XCORR_ERR_INVALID_ARG;
    }
    p.variant = variant;
    if (tile == SUPER_TILE) {
        p.ntile_side = (p.nin + 255) / 256;                // super-rows
        p.tiles_per_chan = p.ntile_side * p.ntile_side;    // triangles + rectangles
    } else {
        p.ntile_side = tile == CHAN_TILE ? 1 : (p.nin + tile - 1) / tile;
        p.tiles_per_chan = p.ntile_side * (p.ntile_side + 1) / 2;
    }

    const bool wide = p.nwindows > 1;
    if (acc == ACC_I8) p.out_dtype = wide ? OUT_CI64 : OUT_CI32;
    else p.out_dtype = wide ? OUT_C128 : OUT_C64;

    const int64_t nbl = (int64_t)nstation * (nstation + 1) / 2;
    p.nitems = (int64_t)nchan * p.tiles_per_chan * p.nwindows;
    p.useful_cmacs = nin64 * (nin64 + 1) / 2 * nchan * (int64_t)ntime;
    p.computed_cmacs = computed_pairs_per_sample(p.nin, tile, acc) * nchan * (int64_t)ntime;
    p.in_bytes = (size_t)ntime * nchan * (size_t)p.nin * in_sample_bytes(in_fmt);
    p.out_bytes = (size_t)nchan * nbl * npol * npol * out_value_bytes(p.out_dtype);
    *pl = p;
    return XCORR_OK;
}

}  // namespace xc
