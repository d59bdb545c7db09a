// C ABI of the X-engine: handles, argument checking, launches.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "plan.h"
#include "xcorr.h"
#include "xeng.h"

using namespace xc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(int e, const char *what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString((hipError_t)e));
    return fail(XCORR_ERR_HIP, buf);
}

constexpr int64_t MAX_BLOCKS_PER_LAUNCH = (1 << 24) - 8;

// Global-load width a kernel may use: whole chunks of `ci` inputs when every row start is
// aligned to the chunk, 32-bit words when rows are word aligned, bytes otherwise.
int load_mode_for(int nin, int in_fmt, int ci)
{
    const int bpc = (int)in_sample_bytes(in_fmt);
    if (nin % ci == 0) return LOAD_VEC;
    if (bpc < 4 && (nin * bpc) % 4 == 0) return LOAD_WORD;
    return LOAD_ELEM;
}

XJob job_from_plan(const Plan &pl, const void *in, void *out)
{
    XJob j;
    memset(&j, 0, sizeof j);
    j.in = in;
    j.out = out;
    j.nin = pl.nin;
    j.npol = pl.npol;
    j.nchan = pl.nchan;
    j.ntime = pl.ntime;
    j.tile = pl.tile;
    j.ntile_side = pl.ntile_side;
    j.tiles_per_chan = pl.tiles_per_chan;
    j.window = pl.window;
    j.nwindows = pl.nwindows;
    j.accumulate = pl.nwindows > 1;
    int ci = 8;
    if (pl.acc == ACC_F32_CMAC) ci = 4;
    else if (pl.acc == ACC_F8 && pl.in_fmt == IN_CI8) ci = 4;
    j.load_mode = load_mode_for(pl.nin, pl.in_fmt, ci);
    j.xcd_group = pl.nchan >= 8 ? 8 : 1;
    j.nitems = pl.nitems;
    const int64_t per_chan = (int64_t)pl.tiles_per_chan * pl.nwindows;
    j.grid = j.xcd_group == 8 ? 8 * ((int64_t)(pl.nchan + 7) / 8) * per_chan : pl.nitems;
    j.block0 = 0;
    return j;
}

// Enqueue one job: zero the output when windows are summed into it, then the tile kernels.
int enqueue_job(const Plan &pl, const void *in, void *out, hipStream_t stream)
{
    if (pl.acc == ACC_F8 && pl.max_abs > 16)
        return fail(XCORR_ERR_UNSUPPORTED, "fp8 e4m3 needs max_abs <= 16 (call xcorr_set_max_abs)");
    // The matrix-core kernels address one block of 64 samples of a channel with 32-bit
    // buffer offsets.
    if (pl.acc != ACC_F32_CMAC &&
        64.0 * (double)pl.nchan * pl.nin * (double)in_sample_bytes(pl.in_fmt) >= 4294901760.0)
        return fail(XCORR_ERR_RANGE, "nchan * nin too large: 64 samples of all channels must span < 4 GiB");
    XJob j = job_from_plan(pl, in, out);
    int e;
    if (pl.nwindows != 1) {
        e = launch_zero(out, pl.out_bytes, stream);
        if (e) return hip_fail(e, "zero fill");
    }
    const int64_t total = j.grid;
    for (int64_t b0 = 0; b0 < total; b0 += MAX_BLOCKS_PER_LAUNCH) {
        j.block0 = b0;
        j.grid = std::min<int64_t>(MAX_BLOCKS_PER_LAUNCH, total - b0);
        e = pl.acc == ACC_F32_CMAC ? launch_cmac(j, pl.in_fmt, stream)
                                   : launch_mfma(j, pl.acc, pl.in_fmt, stream);
        if (e) return hip_fail(e, "kernel launch");
    }
    return XCORR_OK;
}

}  // namespace

struct xcorr_handle {
    Plan plan;
    int device;
};

extern "C" {

const char *xcorr_last_error(void) { return g_err.c_str(); }

int64_t xcorr_window_limit(xcorr_in_dtype in_dtype, xcorr_acc_dtype acc_dtype, int max_abs)
{
    const int64_t w = window_limit((int)in_dtype, (int)acc_dtype, max_abs);
    if (w < 0) return fail(XCORR_ERR_INVALID_ARG, "bad format, path or max_abs");
    return w;
}

int xcorr_tile_coords(int64_t g, int64_t *bx, int64_t *by)
{
    if (g < 0 || !bx || !by) return fail(XCORR_ERR_INVALID_ARG, "g must be >= 0");
    tile_coords(g, bx, by);
    return XCORR_OK;
}

static int plan_info_fill(const Plan &p, xcorr_plan_info *info)
{
    info->nin = p.nin;
    info->tile = p.tile;
    info->ntile_side = p.ntile_side;
    info->tiles_per_chan = p.tiles_per_chan;
    info->window = p.window;
    info->nwindows = p.nwindows;
    info->max_abs = p.max_abs;
    info->out_dtype = p.out_dtype;
    info->nitems = p.nitems;
    info->useful_cmacs = p.useful_cmacs;
    info->computed_cmacs = p.computed_cmacs;
    info->in_bytes = p.in_bytes;
    info->out_bytes = p.out_bytes;
    return XCORR_OK;
}

int xcorr_plan(int nstation, int npol, int nchan, int ntime, xcorr_in_dtype in_dtype,
               xcorr_acc_dtype acc_dtype, int max_abs, xcorr_plan_info *info)
{
    if (!info) return fail(XCORR_ERR_INVALID_ARG, "null info");
    Plan p;
    std::string err;
    const int rc = make_plan(nstation, npol, nchan, ntime, (int)in_dtype, (int)acc_dtype, max_abs, 0, &p, &err);
    if (rc) return fail(rc, err);
    return plan_info_fill(p, info);
}

xcorr_handle_t *xcorr_create(int nstation, int npol, int nchan, int ntime, xcorr_in_dtype in_dtype,
                             xcorr_acc_dtype acc_dtype)
{
    Plan p;
    std::string err;
    // An fp8 job over 8-bit samples is planned with the fp8 bound; runs are refused until
    // the caller declares max_abs <= 16.
    int rc = make_plan(nstation, npol, nchan, ntime, (int)in_dtype, (int)acc_dtype,
                       (acc_dtype == XCORR_ACC_F8E4M3_MMA_F32 && in_dtype == XCORR_IN_CI8) ? 16 : 0, 0,
                       &p, &err);
    if (rc) {
        fail(rc, err);
        return nullptr;
    }
    if (acc_dtype == XCORR_ACC_F8E4M3_MMA_F32 && in_dtype == XCORR_IN_CI8) p.max_abs = 128;
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) {
        hip_fail((int)he, "hipGetDevice");
        return nullptr;
    }
    xcorr_handle *h = new (std::nothrow) xcorr_handle;
    if (!h) {
        fail(XCORR_ERR_OOM, "host allocation");
        return nullptr;
    }
    h->plan = p;
    h->device = dev;
    return h;
}

int xcorr_set_max_abs(xcorr_handle_t *h, int max_abs)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    if (h->plan.in_fmt == IN_CF32) return fail(XCORR_ERR_INVALID_ARG, "max_abs applies to integer samples");
    Plan p;
    std::string err;
    const Plan &o = h->plan;
    const int rc = make_plan(o.nstation, o.npol, o.nchan, o.ntime, o.in_fmt, o.acc, max_abs, o.tile, &p, &err);
    if (rc) return fail(rc, err);
    h->plan = p;
    return XCORR_OK;
}

int xcorr_run(xcorr_handle_t *h, const void *in, void *out, hipStream_t stream)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    if (!out || (!in && h->plan.ntime > 0)) return fail(XCORR_ERR_INVALID_ARG, "null input or output");
    return enqueue_job(h->plan, in, out, stream);
}

void xcorr_destroy(xcorr_handle_t *h) { delete h; }

size_t xcorr_in_bytes(const xcorr_handle_t *h) { return h ? h->plan.in_bytes : 0; }
size_t xcorr_out_bytes(const xcorr_handle_t *h) { return h ? h->plan.out_bytes : 0; }
int xcorr_out_type(const xcorr_handle_t *h)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    return h->plan.out_dtype;
}

}  // extern "C"
