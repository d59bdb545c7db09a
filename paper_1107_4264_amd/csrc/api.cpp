// C ABI of the X-engine: handles, argument checking, launches.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "plan.h"
#include "tune.h"
#include "xcorr.h"
#include "xeng.h"

using namespace xc;

static_assert(NOALLOC_MAX_JOBS == XCORR_NOALLOC_MAX_JOBS, "header and workspace agree on the job limit");
static_assert(NOALLOC_BYTES == XCORR_NOALLOC_SCRATCH_BYTES, "header and workspace agree on the workspace size");

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

// Objects are tied to the device that was current when they were created (their kernels'
// grids, LDS limits and workspace belong to it).
int check_device(int device)
{
    int cur = 0;
    const hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail((int)e, "hipGetDevice");
    if (cur != device)
        return fail(XCORR_ERR_INVALID_ARG, "object created on device " + std::to_string(device) +
                                               " used with device " + std::to_string(cur) + " current");
    return XCORR_OK;
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
    else if ((pl.acc == ACC_F8 || pl.acc == ACC_F6) && pl.in_fmt == IN_CI8) ci = 4;
    j.load_mode = load_mode_for(pl.nin, pl.in_fmt, ci);
    j.xcd_group = pl.nchan >= 8 ? 8 : 1;
    j.staging = pl.staging;
    j.variant = pl.variant;
    j.nitems = pl.nitems;
    const int64_t per_chan = (int64_t)pl.tiles_per_chan * pl.nwindows;
    j.grid = j.xcd_group == 8 ? 8 * ((int64_t)(pl.nchan + 7) / 8) * per_chan : pl.nitems;
    j.block0 = 0;
    return j;
}

// Launch the kernels of one job on `stream` (the output already prepared): the persistent
// whole-channel kernel with one workgroup per compute unit, or one tile kernel launch per
// 2^24 blocks.
int launch_job(const Plan &pl, XJob j, hipStream_t stream)
{
    if (pl.tile == CHAN_TILE || pl.tile == SUPER_TILE) {
        // (fp6 super-tiles need the caller's unit workspace)
        if ((uintptr_t)j.in % 16 == 0 && (pl.tile != SUPER_TILE || pl.acc != ACC_F6 || j.work)) {
            const int cus = device_cus();
            if (cus <= 0) return (int)hipErrorNoDevice;
            if (pl.tile == SUPER_TILE) return launch_super(j, pl.acc, pl.in_fmt, cus, stream);
            j.grid = std::min<int64_t>(pl.nitems, cus);
            return launch_chan(j, pl.acc, stream);
        }
        // the row copies need 16-byte aligned rows (and fp6 super-tiles their workspace): run
        // 128-tiles instead
        Plan tp;
        std::string err;
        if (make_plan(pl.nstation, pl.npol, pl.nchan, pl.ntime, pl.in_fmt, pl.acc, pl.max_abs, 128, &tp, &err,
                      pl.window_req))
            return (int)hipErrorInvalidValue;
        XJob tj = job_from_plan(tp, j.in, j.out);
        tj.accumulate = j.accumulate;
        return launch_job(tp, tj, stream);
    }
    const int64_t total = j.grid;
    for (int64_t b0 = 0; b0 < total; b0 += MAX_BLOCKS_PER_LAUNCH) {
        j.block0 = b0;
        j.grid = std::min<int64_t>(MAX_BLOCKS_PER_LAUNCH, total - b0);
        const int e = pl.acc == ACC_F32_CMAC ? launch_cmac(j, pl.in_fmt, stream)
                      : pl.staging           ? launch_mfma_cache(j, pl.acc, pl.in_fmt, stream)
                                             : launch_mfma(j, pl.acc, pl.in_fmt, stream);
        if (e) return e;
    }
    return 0;
}

// Enqueue one job: zero the output when windows are summed into it, then the tile kernels
// (`work`: the fp6 super-tiles' unit workspace, if any).
int enqueue_job(const Plan &pl, const void *in, void *out, hipStream_t stream, void *work = nullptr)
{
    if (exact_operand_bound(pl.acc) && pl.max_abs > exact_operand_bound(pl.acc))
        return fail(XCORR_ERR_UNSUPPORTED, "fp8 e4m3 needs max_abs <= 16, fp6 e3m2 max_abs <= 8 (call xcorr_set_max_abs)");
    // The matrix-core kernels address one block of 64 samples of a channel with 32-bit
    // buffer offsets.
    if (pl.acc != ACC_F32_CMAC &&
        64.0 * (double)pl.nchan * pl.nin * (double)in_sample_bytes(pl.in_fmt) >= 4294901760.0)
        return fail(XCORR_ERR_RANGE, "nchan * nin too large: 64 samples of all channels must span < 4 GiB");
    XJob j = job_from_plan(pl, in, out);
    j.work = work;
    int e;
    if (pl.nwindows != 1) {
        e = launch_zero(out, pl.out_bytes, stream);
        if (e) return hip_fail(e, "zero fill");
    }
    e = launch_job(pl, j, stream);
    if (e) return hip_fail(e, "kernel launch");
    return XCORR_OK;
}

// Architecture name of the current device ("gfx950"), looked up once per device;
// "unknown" when there is no device.
std::string current_arch()
{
    static std::mutex mu;
    static std::map<int, std::string> names;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    std::lock_guard<std::mutex> lk(mu);
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop;
    std::string name = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        name = prop.gcnArchName;
        const size_t colon = name.find(':');
        if (colon != std::string::npos) name.resize(colon);
        if (name.empty()) name = "unknown";
    }
    names[dev] = name;
    return name;
}

TuneKey key_of(const Plan &p, const std::string &arch)
{
    return TuneKey{arch, p.nstation, p.npol, size_class(p.nchan), size_class(p.ntime), p.in_fmt, p.acc, p.max_abs,
                   p.window_req};
}

// Switch a plan to the kernel shape the autotuner recorded for its class on the current
// device's architecture, if any (and still valid for the job).
void apply_tuned(Plan &p)
{
    TuneVal v;
    if (!tune_lookup(key_of(p, current_arch()), &v)) return;
    if (v.tile == p.tile && v.staging == p.staging && v.variant == p.variant) return;
    Plan q;
    std::string err;
    if (make_plan(p.nstation, p.npol, p.nchan, p.ntime, p.in_fmt, p.acc, p.max_abs, v.tile, &q, &err, p.window_req,
                  v.staging, v.variant) == XCORR_OK) {
        q.max_abs = p.max_abs;
        p = q;
    }
}

}  // namespace

struct xcorr_handle {
    Plan plan;
    int device;
    std::vector<TuneVal> tuned;  // every shape the last xcorr_autotune timed
    bool validate = false;                  // xcorr_run checks the sample range first
    unsigned long long *range_dev = nullptr;  // count of the range check (8 bytes, on first use)
    void *work = nullptr;                     // fp6 super-tiles' unit workspace (on first use)
    size_t work_bytes = 0;
    ~xcorr_handle()
    {
        if (range_dev) (void)hipFree(range_dev);
        if (work) (void)hipFree(work);
    }
};

namespace {

// The unit workspace a plan needs (fp6 super-tiles: f6_work_bytes), allocated on first use
// and grown when a later plan needs more; not inside a graph capture.
int ensure_work(xcorr_handle *h, const Plan &p, hipStream_t stream)
{
    if (p.tile != SUPER_TILE || p.acc != ACC_F6) return XCORR_OK;
    const size_t need = f6_work_bytes(p.nin, p.nchan, p.ntime);
    if (need <= h->work_bytes) return XCORR_OK;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cap);
    if (e != hipSuccess) return hip_fail((int)e, "capture status");
    if (cap != hipStreamCaptureStatusNone)
        return fail(XCORR_ERR_UNSUPPORTED,
                    "the fp6 super-tiles allocate their workspace on the first run: run once before the capture");
    if (h->work) {
        (void)hipFree(h->work);
        h->work = nullptr;
        h->work_bytes = 0;
    }
    e = hipMalloc(&h->work, need);
    if (e != hipSuccess) {
        h->work = nullptr;
        return fail(XCORR_ERR_OOM, "fp6 unit workspace (" + std::to_string(need) + " bytes)");
    }
    h->work_bytes = need;
    return XCORR_OK;
}

}  // namespace

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
               xcorr_acc_dtype acc_dtype, int max_abs, int tile, int window, xcorr_plan_info *info)
{
    if (!info) return fail(XCORR_ERR_INVALID_ARG, "null info");
    Plan p;
    std::string err;
    const int rc =
        make_plan(nstation, npol, nchan, ntime, (int)in_dtype, (int)acc_dtype, max_abs, tile, &p, &err, window);
    if (rc) return fail(rc, err);
    return plan_info_fill(p, info);
}

xcorr_handle_t *xcorr_create(int nstation, int npol, int nchan, int ntime, xcorr_in_dtype in_dtype,
                             xcorr_acc_dtype acc_dtype)
{
    Plan p;
    std::string err;
    // An fp8 / fp6 job over 8-bit samples is planned with the operand type's bound; runs are
    // refused until the caller declares max_abs within it.
    const int lowcap = in_dtype == XCORR_IN_CI8 ? exact_operand_bound((int)acc_dtype) : 0;
    int rc = make_plan(nstation, npol, nchan, ntime, (int)in_dtype, (int)acc_dtype, lowcap, 0, &p, &err);
    if (rc) {
        fail(rc, err);
        return nullptr;
    }
    if (lowcap) p.max_abs = 128;
    apply_tuned(p);
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
    const int rc = make_plan(o.nstation, o.npol, o.nchan, o.ntime, o.in_fmt, o.acc, max_abs, o.tile, &p, &err,
                             o.window_req, o.staging, o.variant);
    if (rc) return fail(rc, err);
    apply_tuned(p);
    h->plan = p;
    return XCORR_OK;
}

int xcorr_autotune(xcorr_handle_t *h, const void *in, void *out, hipStream_t stream, int reps)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    if (!out || (!in && h->plan.ntime > 0)) return fail(XCORR_ERR_INVALID_ARG, "null input or output");
    if (reps < 1 || reps > 1000) return fail(XCORR_ERR_INVALID_ARG, "reps must be in 1..1000");
    if (int rc = check_device(h->device)) return rc;
    const Plan &o = h->plan;
    // every kernel shape the job allows: tile x staging (tiled kernel) x compile-time variant
    std::vector<Plan> cand;
    for (int t : {SUPER_TILE, CHAN_TILE, 128, 64})
        for (int st = 0; st < 2; ++st)
            for (int v = 0; v < kernel_variants(t, o.acc); ++v) {
                Plan q;
                std::string err;
                if (make_plan(o.nstation, o.npol, o.nchan, o.ntime, o.in_fmt, o.acc, o.max_abs, t, &q, &err,
                              o.window_req, st, v) == XCORR_OK) {
                    q.max_abs = o.max_abs;
                    cand.push_back(q);
                }
            }
    if (cand.empty()) return fail(XCORR_ERR_UNSUPPORTED, "no kernel shape accepts this job");
    for (const Plan &q : cand)
        if (int rc = ensure_work(h, q, stream)) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he;
    if ((he = hipEventCreate(&e0)) != hipSuccess || (he = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail((int)he, "autotune events");
    }
    std::vector<TuneVal> timed;
    int best = -1;
    double best_us = 0.0;
    int rc = XCORR_OK;
    // untimed runs first, so that the first shape is not timed while the clocks ramp up
    for (int r = 0; r < reps && rc == XCORR_OK; ++r) rc = enqueue_job(cand[0], in, out, stream, h->work);
    for (size_t c = 0; c < cand.size() && rc == XCORR_OK; ++c) {
        rc = enqueue_job(cand[c], in, out, stream, h->work);  // warm-up
        if (rc) break;
        if ((he = hipEventRecord(e0, stream)) != hipSuccess) {
            rc = hip_fail((int)he, "autotune event");
            break;
        }
        for (int r = 0; r < reps && rc == XCORR_OK; ++r) rc = enqueue_job(cand[c], in, out, stream, h->work);
        if (rc) break;
        float ms = 0.0f;
        if ((he = hipEventRecord(e1, stream)) != hipSuccess || (he = hipEventSynchronize(e1)) != hipSuccess ||
            (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
            rc = hip_fail((int)he, "autotune timing");
            break;
        }
        const double us = 1000.0 * ms / reps;
        timed.push_back(TuneVal{cand[c].tile, cand[c].staging, cand[c].variant, us});
        if (best < 0 || us < best_us) {
            best = (int)c;
            best_us = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    // leave `out` holding the chosen shape's result (bit-identical to every other shape's)
    if ((rc = enqueue_job(cand[best], in, out, stream, h->work)) != XCORR_OK) return rc;
    h->plan = cand[best];
    h->tuned = timed;
    tune_record(key_of(h->plan, current_arch()), TuneVal{h->plan.tile, h->plan.staging, h->plan.variant, best_us});
    return h->plan.tile;
}

int xcorr_autotune_results(const xcorr_handle_t *h, int k, int *tile, int *staging, int *variant, double *us)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    const int n = (int)h->tuned.size();
    if (k >= 0 && k < n) {
        const TuneVal &v = h->tuned[k];
        if (tile) *tile = v.tile;
        if (staging) *staging = v.staging;
        if (variant) *variant = v.variant;
        if (us) *us = v.us;
    }
    return n;
}

int xcorr_autotune_lookup(const char *arch, int nstation, int npol, int nchan, int ntime, xcorr_in_dtype in_dtype,
                          xcorr_acc_dtype acc_dtype, int max_abs, int *staging, int *variant)
{
    Plan p;
    std::string err;
    const int rc = make_plan(nstation, npol, nchan, ntime, (int)in_dtype, (int)acc_dtype, max_abs, 0, &p, &err);
    if (rc) return fail(rc, err);
    TuneVal v;
    if (!tune_lookup(key_of(p, arch ? std::string(arch) : current_arch()), &v)) return 0;
    if (staging) *staging = v.staging;
    if (variant) *variant = v.variant;
    return v.tile;
}

int xcorr_autotune_save(const char *path)
{
    if (!path) return fail(XCORR_ERR_INVALID_ARG, "null path");
    std::string err;
    const int n = tune_save(path, &err);
    return n < 0 ? fail(XCORR_ERR_INVALID_ARG, err) : n;
}

int xcorr_autotune_load(const char *path)
{
    if (!path) return fail(XCORR_ERR_INVALID_ARG, "null path");
    std::string err;
    const int n = tune_load(path, &err);
    return n < 0 ? fail(XCORR_ERR_INVALID_ARG, err) : n;
}

void xcorr_autotune_clear(void) { tune_clear(); }

int xcorr_set_tile(xcorr_handle_t *h, int tile)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    Plan p;
    std::string err;
    const Plan &o = h->plan;
    const int rc = make_plan(o.nstation, o.npol, o.nchan, o.ntime, o.in_fmt, o.acc, o.max_abs, tile, &p, &err,
                             o.window_req, o.staging, 0);
    if (rc) return fail(rc, err);
    h->plan = p;
    return XCORR_OK;
}

int xcorr_set_staging(xcorr_handle_t *h, int staging)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    Plan p;
    std::string err;
    const Plan &o = h->plan;
    // keep a tiled kernel's tile; the whole-channel and super-tiled kernels always stage
    // in LDS, so caching through L1 / L2 falls back to the automatic tile
    const int tile = (o.tile == 64 || o.tile == 128) ? o.tile : 0;
    const int rc = make_plan(o.nstation, o.npol, o.nchan, o.ntime, o.in_fmt, o.acc, o.max_abs, staging ? tile : 0, &p,
                             &err, o.window_req, staging, 0);
    if (rc) return fail(rc, err);
    h->plan = p;
    return XCORR_OK;
}

int xcorr_get_staging(const xcorr_handle_t *h)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    return h->plan.staging;
}

int xcorr_set_variant(xcorr_handle_t *h, int variant)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    Plan p;
    std::string err;
    const Plan &o = h->plan;
    const int rc = make_plan(o.nstation, o.npol, o.nchan, o.ntime, o.in_fmt, o.acc, o.max_abs, o.tile, &p, &err,
                             o.window_req, o.staging, variant);
    if (rc) return fail(rc, err);
    h->plan = p;
    return XCORR_OK;
}

int xcorr_get_variant(const xcorr_handle_t *h)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    return h->plan.variant;
}

int xcorr_set_window(xcorr_handle_t *h, int window)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    Plan p;
    std::string err;
    const Plan &o = h->plan;
    // an fp8 job over 8-bit samples without a declared bound plans with the fp8 bound and
    // stays refused at run time (see xcorr_create)
    const int cap = exact_operand_bound(o.acc);
    const bool undeclared = cap && o.in_fmt == IN_CI8 && o.max_abs > cap;
    const int ma = undeclared ? cap : o.max_abs;
    // keep a tile the caller or the autotuner chose, unless the new windows rule it out
    int rc = make_plan(o.nstation, o.npol, o.nchan, o.ntime, o.in_fmt, o.acc, ma, o.tile, &p, &err, window, o.staging,
                       o.variant);
    if (rc == XCORR_ERR_INVALID_ARG && window >= 0)
        rc = make_plan(o.nstation, o.npol, o.nchan, o.ntime, o.in_fmt, o.acc, ma, 0, &p, &err, window, o.staging, 0);
    if (rc) return fail(rc, err);
    if (undeclared) p.max_abs = o.max_abs;
    h->plan = p;
    return XCORR_OK;
}

int xcorr_get_tile(const xcorr_handle_t *h)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    return h->plan.tile;
}

int xcorr_validate(xcorr_handle_t *h, const void *in, hipStream_t stream, int64_t *nbad)
{
    if (!h || !nbad) return fail(XCORR_ERR_INVALID_ARG, "null handle or count");
    const Plan &p = h->plan;
    if (!in && p.in_bytes > 0) return fail(XCORR_ERR_INVALID_ARG, "null input");
    if (int rc = check_device(h->device)) return rc;
    *nbad = 0;
    if (p.in_fmt == IN_CF32 || p.in_bytes == 0) return XCORR_OK;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cap);
    if (e != hipSuccess) return hip_fail((int)e, "capture status");
    if (cap != hipStreamCaptureStatusNone)
        return fail(XCORR_ERR_UNSUPPORTED, "the range check waits for its result: not inside a graph capture");
    if (!h->range_dev) {
        e = hipMalloc((void **)&h->range_dev, sizeof(unsigned long long));
        if (e != hipSuccess) {
            h->range_dev = nullptr;
            return fail(XCORR_ERR_OOM, "range-check counter");
        }
    }
    if (int rc = launch_range_count(in, p.in_bytes, p.in_fmt == IN_CI4, p.max_abs, h->range_dev, stream))
        return hip_fail(rc, "range check");
    unsigned long long n = 0;
    e = hipMemcpyAsync(&n, h->range_dev, sizeof n, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail((int)e, "range-check result");
    *nbad = (int64_t)n;
    return XCORR_OK;
}

int xcorr_set_validation(xcorr_handle_t *h, int on)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    if (on != 0 && on != 1) return fail(XCORR_ERR_INVALID_ARG, "validation is 0 (off) or 1 (on)");
    h->validate = on == 1;
    return XCORR_OK;
}

int xcorr_run(xcorr_handle_t *h, const void *in, void *out, hipStream_t stream)
{
    if (!h) return fail(XCORR_ERR_INVALID_ARG, "null handle");
    if (!out || (!in && h->plan.ntime > 0)) return fail(XCORR_ERR_INVALID_ARG, "null input or output");
    if (int rc = check_device(h->device)) return rc;
    if (h->validate) {
        int64_t nbad = 0;
        if (int rc = xcorr_validate(h, in, stream, &nbad)) return rc;
        if (nbad)
            return fail(XCORR_ERR_RANGE, std::to_string(nbad) + " sample components outside [-" +
                                             std::to_string(h->plan.max_abs) + ", " +
                                             std::to_string(h->plan.max_abs) + "]: nothing computed");
    }
    if (int rc = ensure_work(h, h->plan, stream)) return rc;
    return enqueue_job(h->plan, in, out, stream, h->work);
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

// ------------------------------------------------------------------ batches

struct xcorr_batch {
    int device = 0;
    int in_fmt = 0, acc = 0, tile = 0, mode = 0;
    int cus = 0;
    std::vector<xcorr_job> jobs;
    std::vector<Plan> plans;
    std::vector<char> whole;  // job runs the whole-channel kernel (its own persistent launch)
    XQueues queues{};
    int64_t nitems = 0;
    XItem *items_dev = nullptr;
    XJob *jobs_dev = nullptr;
    XJob *jobs_pinned = nullptr;
    unsigned int *counters_dev = nullptr;
    hipEvent_t uploaded = nullptr;
    bool upload_pending = false;
};

namespace {

void batch_free(xcorr_batch *b)
{
    if (!b) return;
    if (b->items_dev) (void)hipFree(b->items_dev);
    if (b->jobs_dev) (void)hipFree(b->jobs_dev);
    if (b->counters_dev) (void)hipFree(b->counters_dev);
    if (b->jobs_pinned) (void)hipHostFree(b->jobs_pinned);
    if (b->uploaded) (void)hipEventDestroy(b->uploaded);
    delete b;
}

// Plan every job with a common tile and load mode, build the queues of work items and
// upload them.  Items of one (job, channel) share a queue, so on the XCD that owns the
// queue the tiles re-reading that channel's inputs share an L2; each queue is ordered
// longest item first.
// Common tile of a batch's tiled launch: 64 for the FP32 CMAC path and for arrays of at
// most 64 inputs, 128 otherwise.
int batch_tile(const xcorr_job *jobs, int njobs, int acc)
{
    int max_nin = 0;
    for (int j = 0; j < njobs; ++j) max_nin = std::max(max_nin, jobs[j].nstation * jobs[j].npol);
    return acc == ACC_F32_CMAC ? 64 : (max_nin > 64 ? 128 : 64);
}

// Plan job `idx` of a batch: with the batch's common tile, or with its own whole-channel or
// super-tiled plan when the planner gives it one (*whole = 1: it runs its own persistent
// launch).  max_abs 0: the format's default.
int plan_batch_job(const xcorr_job &jb, int idx, int in_fmt, int acc, int max_abs, int tile, Plan *pl, char *whole)
{
    std::string err;
    int ma = max_abs;
    const int cap = in_fmt == IN_CI8 ? exact_operand_bound(acc) : 0;
    if (cap && ma == 0) ma = cap;  // runs refused until declared
    const int rc = make_plan(jb.nstation, jb.npol, jb.nchan, jb.ntime, in_fmt, acc, ma, tile, pl, &err);
    if (rc) return fail(rc, "job " + std::to_string(idx) + ": " + err);
    if (cap && max_abs == 0) pl->max_abs = 128;
    *whole = 0;
    Plan wp;
    if (acc != ACC_F32_CMAC && make_plan(jb.nstation, jb.npol, jb.nchan, jb.ntime, in_fmt, acc, ma, 0, &wp, &err) == XCORR_OK &&
        (wp.tile == CHAN_TILE || wp.tile == SUPER_TILE)) {
        wp.max_abs = pl->max_abs;
        *pl = wp;
        *whole = 1;
    }
    if (acc != ACC_F32_CMAC && 64.0 * (double)jb.nchan * pl->nin * (double)in_sample_bytes(in_fmt) >= 4294901760.0)
        return fail(XCORR_ERR_RANGE, "job " + std::to_string(idx) + ": nchan * nin too large");
    return XCORR_OK;
}

// Plan every job with a common tile and load mode, build the queues of work items and
// upload them.  Items of one (job, channel) share a queue, so on the XCD that owns the
// queue the tiles re-reading that channel's inputs share an L2; each queue is ordered
// longest item first.
int batch_plan(xcorr_batch *b, int max_abs)
{
    const int njobs = (int)b->jobs.size();
    const int tile = batch_tile(b->jobs.data(), njobs, b->acc);
    std::vector<Plan> plans(njobs);
    std::vector<char> whole(njobs, 0);
    int ci = b->acc == ACC_F32_CMAC ? 4 : ((exact_operand_bound(b->acc) && b->in_fmt == IN_CI8) ? 4 : 8);
    int mode = LOAD_VEC;
    for (int j = 0; j < njobs; ++j) {
        if (int rc = plan_batch_job(b->jobs[j], j, b->in_fmt, b->acc, max_abs, tile, &plans[j], &whole[j])) return rc;
        if (!whole[j]) mode = std::max(mode, load_mode_for(plans[j].nin, b->in_fmt, ci));
    }
    // Work items in groups of one (job, channel, window): the tiles of a group read the same
    // input rows, so they stay adjacent in their queue (taken at about the same time by
    // workgroups of one XCD, whose L2 then serves the re-reads).  Groups are ordered longest
    // first (cost: computed pairs x samples).
    struct Group {
        double cost;
        std::vector<XItem> items;
    };
    std::vector<std::vector<Group>> q(NQUEUE);
    for (int j = 0; j < njobs; ++j) {
        const Plan &pl = plans[j];
        if (whole[j]) continue;
        for (int f = 0; f < pl.nchan; ++f) {
            const int qq = (int)(((int64_t)j * 131 + f) % NQUEUE);
            for (int w = 0; w < pl.nwindows; ++w) {
                const int len = std::min(pl.ntime - w * pl.window, pl.window);
                Group gr{0.0, {}};
                for (int g = 0; g < pl.tiles_per_chan; ++g) {
                    int64_t bx, by;
                    tile_coords(g, &bx, &by);
                    const int rows = std::min(pl.tile, pl.nin - (int)by * pl.tile);
                    const int cols = std::min(pl.tile, pl.nin - (int)bx * pl.tile);
                    double c = (double)rows * cols * len;
                    if (bx == by && b->acc != ACC_F32_CMAC) c *= 0.625;  // lower 32x32 blocks only
                    gr.cost += c;
                    gr.items.push_back(XItem{j, f, g, w});
                }
                q[qq].push_back(std::move(gr));
            }
        }
    }
    std::vector<XItem> items;
    XQueues qs{};
    for (int k = 0; k < NQUEUE; ++k) {
        std::stable_sort(q[k].begin(), q[k].end(), [](const Group &a, const Group &c) { return a.cost > c.cost; });
        qs.begin[k] = (int64_t)items.size();
        for (const Group &gr : q[k]) items.insert(items.end(), gr.items.begin(), gr.items.end());
        qs.end[k] = (int64_t)items.size();
    }
    if (b->items_dev) {
        (void)hipFree(b->items_dev);
        b->items_dev = nullptr;
    }
    if (!items.empty()) {
        hipError_t e = hipMalloc(&b->items_dev, items.size() * sizeof(XItem));
        if (e != hipSuccess) return hip_fail((int)e, "hipMalloc work list");
        e = hipMemcpy(b->items_dev, items.data(), items.size() * sizeof(XItem), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail((int)e, "upload work list");
    }
    b->plans = plans;
    b->whole = whole;
    b->tile = tile;
    b->mode = mode;
    b->queues = qs;
    b->nitems = (int64_t)items.size();
    b->cus = std::max(1, device_cus());
    return XCORR_OK;
}

}  // namespace

extern "C" {

xcorr_batch_t *xcorr_batch_create(int njobs, const xcorr_job *jobs, xcorr_in_dtype in_dtype,
                                  xcorr_acc_dtype acc_dtype)
{
    if (njobs < 1 || !jobs) {
        fail(XCORR_ERR_INVALID_ARG, "need njobs >= 1 and a job array");
        return nullptr;
    }
    xcorr_batch *b = new (std::nothrow) xcorr_batch;
    if (!b) {
        fail(XCORR_ERR_OOM, "host allocation");
        return nullptr;
    }
    b->in_fmt = (int)in_dtype;
    b->acc = (int)acc_dtype;
    b->jobs.assign(jobs, jobs + njobs);
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        hip_fail((int)e, "hipGetDevice");
        batch_free(b);
        return nullptr;
    }
    if (batch_plan(b, 0) != XCORR_OK) {
        batch_free(b);
        return nullptr;
    }
    if ((e = hipMalloc(&b->jobs_dev, njobs * sizeof(XJob))) != hipSuccess ||
        (e = hipMalloc(&b->counters_dev, NQUEUE * COUNTER_STRIDE * sizeof(unsigned int))) != hipSuccess ||
        (e = hipHostMalloc(&b->jobs_pinned, njobs * sizeof(XJob), hipHostMallocDefault)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming)) != hipSuccess) {
        hip_fail((int)e, "batch allocation");
        batch_free(b);
        return nullptr;
    }
    return b;
}

int xcorr_batch_set_max_abs(xcorr_batch_t *b, int max_abs)
{
    if (!b) return fail(XCORR_ERR_INVALID_ARG, "null batch");
    if (b->in_fmt == IN_CF32) return fail(XCORR_ERR_INVALID_ARG, "max_abs applies to integer samples");
    if (max_abs < 1) return fail(XCORR_ERR_INVALID_ARG, "max_abs must be >= 1");
    return batch_plan(b, max_abs);
}

int xcorr_batch_run(xcorr_batch_t *b, const void *const *in, void *const *out, hipStream_t stream)
{
    if (!b || !in || !out) return fail(XCORR_ERR_INVALID_ARG, "null batch or pointer array");
    const int njobs = (int)b->jobs.size();
    if (exact_operand_bound(b->acc) && b->plans[0].max_abs > exact_operand_bound(b->acc))
        return fail(XCORR_ERR_UNSUPPORTED,
                    "fp8 e4m3 needs max_abs <= 16, fp6 e3m2 max_abs <= 8 (call xcorr_batch_set_max_abs)");
    for (int j = 0; j < njobs; ++j)
        if (!out[j] || (!in[j] && b->plans[j].ntime > 0))
            return fail(XCORR_ERR_INVALID_ARG, "null input or output of job " + std::to_string(j));
    if (int rc = check_device(b->device)) return rc;
    hipError_t e;
    if (b->upload_pending) {
        // the pinned table is still being read by the previous run's copy
        if ((e = hipEventSynchronize(b->uploaded)) != hipSuccess) return hip_fail((int)e, "batch table event");
        b->upload_pending = false;
    }
    for (int j = 0; j < njobs; ++j) {
        XJob jb = job_from_plan(b->plans[j], in[j], out[j]);
        jb.load_mode = b->mode;  // the launch's mode covers every job
        b->jobs_pinned[j] = jb;
    }
    if ((e = hipMemcpyAsync(b->jobs_dev, b->jobs_pinned, njobs * sizeof(XJob), hipMemcpyHostToDevice, stream)) !=
        hipSuccess)
        return hip_fail((int)e, "batch table upload");
    if ((e = hipEventRecord(b->uploaded, stream)) != hipSuccess) return hip_fail((int)e, "batch table event");
    b->upload_pending = true;
    int rc = launch_zero(b->counters_dev, NQUEUE * COUNTER_STRIDE * sizeof(unsigned int), stream);
    if (rc) return hip_fail(rc, "zero counters");
    for (int j = 0; j < njobs; ++j)
        if (b->plans[j].nwindows != 1) {
            rc = launch_zero(out[j], b->plans[j].out_bytes, stream);
            if (rc) return hip_fail(rc, "zero fill");
        }
    for (int j = 0; j < njobs; ++j)
        if (b->whole[j]) {
            rc = launch_job(b->plans[j], job_from_plan(b->plans[j], in[j], out[j]), stream);
            if (rc) return hip_fail(rc, "whole-channel / super-tile launch of a batch job");
        }
    if (b->nitems == 0) return XCORR_OK;
    // persistent workgroups: as many as fit the compute units at once
    int64_t nblocks = (int64_t)b->cus * (b->acc == ACC_F32_CMAC ? 4 : 2);
    nblocks = std::max<int64_t>(1, std::min(nblocks, b->nitems));
    rc = b->acc == ACC_F32_CMAC
             ? launch_cmac_batch(b->jobs_dev, b->items_dev, b->queues, b->counters_dev, b->in_fmt, (int)nblocks, stream)
             : launch_mfma_batch(b->jobs_dev, b->items_dev, b->queues, b->counters_dev, b->acc, b->in_fmt, b->tile,
                                 b->mode, (int)nblocks, stream);
    if (rc) return hip_fail(rc, "batch kernel launch");
    return XCORR_OK;
}

size_t xcorr_batch_in_bytes(const xcorr_batch_t *b, int job)
{
    return (b && job >= 0 && job < (int)b->plans.size()) ? b->plans[job].in_bytes : 0;
}

size_t xcorr_batch_out_bytes(const xcorr_batch_t *b, int job)
{
    return (b && job >= 0 && job < (int)b->plans.size()) ? b->plans[job].out_bytes : 0;
}

int xcorr_batch_out_type(const xcorr_batch_t *b, int job)
{
    if (!b || job < 0 || job >= (int)b->plans.size()) return fail(XCORR_ERR_INVALID_ARG, "bad batch or job");
    return b->plans[job].out_dtype;
}

int64_t xcorr_batch_items(const xcorr_batch_t *b) { return b ? b->nitems : 0; }

void xcorr_batch_destroy(xcorr_batch_t *b)
{
    if (!b) return;
    if (b->upload_pending) (void)hipEventSynchronize(b->uploaded);
    batch_free(b);
}

int xcorr_batch_run_noalloc(int njobs, const xcorr_job *jobs, xcorr_in_dtype in_dtype, xcorr_acc_dtype acc_dtype,
                            int max_abs, const void *const *in, void *const *out, hipStream_t stream)
{
    if (njobs < 1 || !jobs || !in || !out) return fail(XCORR_ERR_INVALID_ARG, "need njobs >= 1 and the job, input and output arrays");
    if (njobs > NOALLOC_MAX_JOBS)
        return fail(XCORR_ERR_INVALID_ARG, "xcorr_batch_run_noalloc takes at most " + std::to_string(NOALLOC_MAX_JOBS) +
                                               " jobs (its workspace is fixed)");
    const int in_fmt = (int)in_dtype, acc = (int)acc_dtype;
    if (max_abs < 0) return fail(XCORR_ERR_INVALID_ARG, "max_abs must be >= 0 (0: the format's default)");
    if (in_fmt == IN_CF32 && max_abs != 0) return fail(XCORR_ERR_INVALID_ARG, "max_abs applies to integer samples");
    if (exact_operand_bound(acc) && in_fmt == IN_CI8 && (max_abs == 0 || max_abs > exact_operand_bound(acc)))
        return fail(XCORR_ERR_UNSUPPORTED,
                    "fp8 e4m3 / fp6 e3m2 need a declared max_abs <= 16 / 8 for 8-bit samples");
    // Host planning in fixed arrays: nothing is allocated on the host or the device.
    const int tile = batch_tile(jobs, njobs, acc);
    const int ci = acc == ACC_F32_CMAC ? 4 : ((exact_operand_bound(acc) && in_fmt == IN_CI8) ? 4 : 8);
    Plan plans[NOALLOC_MAX_JOBS];
    char whole[NOALLOC_MAX_JOBS];
    int mode = LOAD_VEC;
    for (int j = 0; j < njobs; ++j) {
        if (int rc = plan_batch_job(jobs[j], j, in_fmt, acc, max_abs, tile, &plans[j], &whole[j])) return rc;
        if (!whole[j]) mode = std::max(mode, load_mode_for(plans[j].nin, in_fmt, ci));
        if (!out[j] || (!in[j] && plans[j].ntime > 0))
            return fail(XCORR_ERR_INVALID_ARG, "null input or output of job " + std::to_string(j));
    }
    void *ws = nullptr;
    if (int e = noalloc_scratch(&ws)) return hip_fail(e, "workspace address");
    for (int j = 0; j < njobs; ++j)
        if (plans[j].nwindows != 1)
            if (int rc = launch_zero(out[j], plans[j].out_bytes, stream)) return hip_fail(rc, "zero fill");
    for (int j = 0; j < njobs; ++j)
        if (whole[j])
            if (int rc = launch_job(plans[j], job_from_plan(plans[j], in[j], out[j]), stream))
                return hip_fail(rc, "whole-channel / super-tile launch of a batch job");
    // The other jobs share one persistent launch of the tiled kernel over a work list the
    // kernel generates from the job table (longest items first).
    int order[NOALLOC_MAX_JOBS];
    int ntab = 0;
    for (int j = 0; j < njobs; ++j)
        if (!whole[j] && plans[j].nitems > 0) order[ntab++] = j;
    if (ntab == 0) return XCORR_OK;
    auto item_cost = [&](int j) {
        const double side = std::min(plans[j].nin, tile);
        return (double)plans[j].window * side * side;
    };
    std::sort(order, order + ntab, [&](int a, int c) {
        const double ca = item_cost(a), cc = item_cost(c);
        return ca > cc || (ca == cc && a < c);
    });
    XJob table[NOALLOC_MAX_JOBS];
    int64_t total = 0;
    for (int k = 0; k < ntab; ++k) {
        const int j = order[k];
        XJob jb = job_from_plan(plans[j], in[j], out[j]);
        jb.load_mode = mode;  // the launch's mode covers every job
        table[k] = jb;
        total += plans[j].nitems;
    }
    if (int rc = launch_noalloc_setup(ws, table, ntab, stream)) return hip_fail(rc, "workspace set-up");
    uint8_t *w = (uint8_t *)ws;
    const XGenQueues g{(const int64_t *)(w + NOALLOC_QEND_OFF), ntab, NOALLOC_MAX_JOBS};
    const XJob *jobs_dev = (const XJob *)(w + NOALLOC_JOBS_OFF);
    unsigned int *counters = (unsigned int *)(w + NOALLOC_COUNTERS_OFF);
    int nblocks = std::max(1, device_cus()) * (acc == ACC_F32_CMAC ? 4 : 2);
    if ((int64_t)nblocks > total) nblocks = (int)total;
    const int rc = acc == ACC_F32_CMAC
                       ? launch_cmac_batch_gen(jobs_dev, g, counters, in_fmt, nblocks, stream)
                       : launch_mfma_batch_gen(jobs_dev, g, counters, acc, in_fmt, tile, mode, nblocks, stream);
    if (rc) return hip_fail(rc, "batch kernel launch");
    return XCORR_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ streaming integration

struct xcorr_stream {
    Plan plan;  // one chunk
    int device = 0;
    hipStream_t copy_stream = nullptr;
    void *dbuf[2] = {nullptr, nullptr};
    hipEvent_t copied[2] = {nullptr, nullptr};
    hipEvent_t consumed[2] = {nullptr, nullptr};
    hipEvent_t began = nullptr;
    bool consumed_valid[2] = {false, false};
    bool copied_valid[2] = {false, false};  // copied[k] records an eager (not captured) copy
    void *out = nullptr;
    int64_t npush = 0;
};

namespace {

void stream_free(xcorr_stream *s)
{
    if (!s) return;
    if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
    for (int k = 0; k < 2; ++k) {
        if (s->dbuf[k]) (void)hipFree(s->dbuf[k]);
        if (s->copied[k]) (void)hipEventDestroy(s->copied[k]);
        if (s->consumed[k]) (void)hipEventDestroy(s->consumed[k]);
    }
    if (s->began) (void)hipEventDestroy(s->began);
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    delete s;
}

// Wide totals: the output type of a multi-window run.
int wide_type(int acc) { return acc == ACC_I8 ? OUT_CI64 : OUT_C128; }

}  // namespace

extern "C" {

xcorr_stream_t *xcorr_stream_create(int nstation, int npol, int nchan, int chunk_ntime, xcorr_in_dtype in_dtype,
                                    xcorr_acc_dtype acc_dtype)
{
    if (chunk_ntime < 1) {
        fail(XCORR_ERR_INVALID_ARG, "chunk_ntime must be >= 1");
        return nullptr;
    }
    xcorr_stream *s = new (std::nothrow) xcorr_stream;
    if (!s) {
        fail(XCORR_ERR_OOM, "host allocation");
        return nullptr;
    }
    std::string err;
    const int lowcap = in_dtype == XCORR_IN_CI8 ? exact_operand_bound((int)acc_dtype) : 0;
    int rc = make_plan(nstation, npol, nchan, chunk_ntime, (int)in_dtype, (int)acc_dtype, lowcap, 0, &s->plan, &err);
    if (rc) {
        fail(rc, err);
        delete s;
        return nullptr;
    }
    if (lowcap) s->plan.max_abs = 128;
    if (s->plan.acc != ACC_F32_CMAC &&
        64.0 * (double)nchan * s->plan.nin * (double)in_sample_bytes(s->plan.in_fmt) >= 4294901760.0) {
        fail(XCORR_ERR_RANGE, "nchan * nin too large: 64 samples of all channels must span < 4 GiB");
        delete s;
        return nullptr;
    }
    hipError_t e;
    if ((e = hipGetDevice(&s->device)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&s->began, hipEventDisableTiming)) != hipSuccess) {
        hip_fail((int)e, "stream setup");
        stream_free(s);
        return nullptr;
    }
    for (int k = 0; k < 2; ++k) {
        if ((e = hipMalloc(&s->dbuf[k], std::max<size_t>(s->plan.in_bytes, 16))) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s->copied[k], hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&s->consumed[k], hipEventDisableTiming)) != hipSuccess) {
            hip_fail((int)e, "stream buffers");
            stream_free(s);
            return nullptr;
        }
    }
    return s;
}

int xcorr_stream_set_max_abs(xcorr_stream_t *s, int max_abs)
{
    if (!s) return fail(XCORR_ERR_INVALID_ARG, "null stream object");
    if (s->out) return fail(XCORR_ERR_INVALID_ARG, "an integration is in progress");
    if (s->plan.in_fmt == IN_CF32) return fail(XCORR_ERR_INVALID_ARG, "max_abs applies to integer samples");
    Plan p;
    std::string err;
    const Plan &o = s->plan;
    const int rc = make_plan(o.nstation, o.npol, o.nchan, o.ntime, o.in_fmt, o.acc, max_abs, o.tile, &p, &err,
                             o.window_req);
    if (rc) return fail(rc, err);
    s->plan = p;
    return XCORR_OK;
}

int xcorr_stream_set_window(xcorr_stream_t *s, int window)
{
    if (!s) return fail(XCORR_ERR_INVALID_ARG, "null stream object");
    if (s->out) return fail(XCORR_ERR_INVALID_ARG, "an integration is in progress");
    Plan p;
    std::string err;
    const Plan &o = s->plan;
    const int cap = exact_operand_bound(o.acc);
    const bool undeclared = cap && o.in_fmt == IN_CI8 && o.max_abs > cap;
    const int ma = undeclared ? cap : o.max_abs;
    const int rc = make_plan(o.nstation, o.npol, o.nchan, o.ntime, o.in_fmt, o.acc, ma, 0, &p, &err, window);
    if (rc) return fail(rc, err);
    if (undeclared) p.max_abs = o.max_abs;
    s->plan = p;
    return XCORR_OK;
}

int xcorr_stream_begin(xcorr_stream_t *s, void *out, hipStream_t stream)
{
    if (!s || !out) return fail(XCORR_ERR_INVALID_ARG, "null stream object or output");
    if (int rc = check_device(s->device)) return rc;
    if (exact_operand_bound(s->plan.acc) && s->plan.max_abs > exact_operand_bound(s->plan.acc))
        return fail(XCORR_ERR_UNSUPPORTED,
                    "fp8 e4m3 needs max_abs <= 16, fp6 e3m2 max_abs <= 8 (call xcorr_stream_set_max_abs)");
    Plan wide = s->plan;
    wide.out_dtype = wide_type(wide.acc);
    wide.out_bytes = s->plan.out_bytes / out_value_bytes(s->plan.out_dtype) * out_value_bytes(wide.out_dtype);
    int rc = launch_zero(out, wide.out_bytes, stream);
    if (rc) return hip_fail(rc, "zero totals");
    hipError_t e = hipEventRecord(s->began, stream);
    if (e != hipSuccess) return hip_fail((int)e, "stream begin event");
    s->out = out;
    s->npush = 0;
    s->consumed_valid[0] = s->consumed_valid[1] = false;
    s->copied_valid[0] = s->copied_valid[1] = false;
    return XCORR_OK;
}

int xcorr_stream_push(xcorr_stream_t *s, const void *host_chunk, hipStream_t stream)
{
    if (!s || !host_chunk) return fail(XCORR_ERR_INVALID_ARG, "null stream object or chunk");
    if (!s->out) return fail(XCORR_ERR_INVALID_ARG, "xcorr_stream_begin was not called");
    const int slot = (int)(s->npush & 1);
    hipError_t e;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if ((e = hipStreamIsCapturing(stream, &cap)) != hipSuccess) return hip_fail((int)e, "capture status");
    const bool eager = cap == hipStreamCaptureStatusNone;
    // Release point of the host chunks: push p waits on the host for the copy of chunk
    // p - 2 (the last copy through this slot), so once push p returns the caller may reuse
    // chunk p - 2 (Algorithm 1 synchronises every iteration for the same reason).  The copy
    // queue is one chunk deep by then, so the wait costs no overlap.  Copies recorded into a
    // graph are not waited for here (each launch of the graph orders its own copies).
    if (eager && s->copied_valid[slot]) {
        if ((e = hipEventSynchronize(s->copied[slot])) != hipSuccess) return hip_fail((int)e, "chunk release wait");
        s->copied_valid[slot] = false;
    }
    // the copy into this buffer waits for the kernel that last read it (or for the start
    // of the integration); the kernel waits for the copy
    e = hipStreamWaitEvent(s->copy_stream, s->consumed_valid[slot] ? s->consumed[slot] : s->began, 0);
    if (e != hipSuccess) return hip_fail((int)e, "copy wait");
    if (s->plan.in_bytes) {
        e = hipMemcpyAsync(s->dbuf[slot], host_chunk, s->plan.in_bytes, hipMemcpyHostToDevice, s->copy_stream);
        if (e != hipSuccess) return hip_fail((int)e, "chunk copy");
    }
    if ((e = hipEventRecord(s->copied[slot], s->copy_stream)) != hipSuccess) return hip_fail((int)e, "copy event");
    s->copied_valid[slot] = eager;
    if ((e = hipStreamWaitEvent(stream, s->copied[slot], 0)) != hipSuccess) return hip_fail((int)e, "compute wait");
    XJob j = job_from_plan(s->plan, s->dbuf[slot], s->out);
    j.accumulate = 1;  // add into the wide totals
    const int rc = launch_job(s->plan, j, stream);
    if (rc) return hip_fail(rc, "kernel launch");
    if ((e = hipEventRecord(s->consumed[slot], stream)) != hipSuccess) return hip_fail((int)e, "compute event");
    s->consumed_valid[slot] = true;
    s->npush += 1;
    return XCORR_OK;
}

int64_t xcorr_stream_end(xcorr_stream_t *s, hipStream_t stream)
{
    (void)stream;  // every chunk's kernel already runs on `stream`, after its copy
    if (!s) return fail(XCORR_ERR_INVALID_ARG, "null stream object");
    if (!s->out) return fail(XCORR_ERR_INVALID_ARG, "xcorr_stream_begin was not called");
    s->out = nullptr;
    return s->npush * (int64_t)s->plan.ntime;
}

size_t xcorr_stream_chunk_bytes(const xcorr_stream_t *s) { return s ? s->plan.in_bytes : 0; }

size_t xcorr_stream_out_bytes(const xcorr_stream_t *s)
{
    if (!s) return 0;
    return s->plan.out_bytes / out_value_bytes(s->plan.out_dtype) * out_value_bytes(wide_type(s->plan.acc));
}

int xcorr_stream_out_type(const xcorr_stream_t *s)
{
    if (!s) return fail(XCORR_ERR_INVALID_ARG, "null stream object");
    return wide_type(s->plan.acc);
}

void xcorr_stream_destroy(xcorr_stream_t *s) { stream_free(s); }

int xcorr_stream_capture(xcorr_stream_t *s, int nchunk, const void *const *host_chunks, void *out,
                         hipGraphExec_t *exec)
{
    if (!s || !exec || !out || nchunk < 1 || !host_chunks)
        return fail(XCORR_ERR_INVALID_ARG, "null argument or nchunk < 1");
    for (int c = 0; c < nchunk; ++c)
        if (!host_chunks[c]) return fail(XCORR_ERR_INVALID_ARG, "null chunk");
    *exec = nullptr;
    hipStream_t cs = nullptr;
    hipError_t he = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (he != hipSuccess) return hip_fail((int)he, "capture stream");
    // relaxed mode: the first launch of a kernel may set its LDS limit while capturing
    he = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (he != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail((int)he, "begin capture");
    }
    int rc = xcorr_stream_begin(s, out, cs);
    for (int c = 0; c < nchunk && rc == XCORR_OK; ++c) rc = xcorr_stream_push(s, host_chunks[c], cs);
    if (rc == XCORR_OK) {
        const int64_t n = xcorr_stream_end(s, cs);
        if (n < 0) rc = (int)n;
    } else {
        s->out = nullptr;
    }
    // end the capture in every case; a failure above keeps its own message
    hipGraph_t g = nullptr;
    he = hipStreamEndCapture(cs, &g);
    if (rc == XCORR_OK && he != hipSuccess) rc = hip_fail((int)he, "end capture");
    if (rc == XCORR_OK) {
        he = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
        if (he != hipSuccess) rc = hip_fail((int)he, "instantiate graph");
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    if (rc != XCORR_OK) *exec = nullptr;
    return rc;
}

int xcorr_graph_launch(hipGraphExec_t exec, hipStream_t stream)
{
    if (!exec) return fail(XCORR_ERR_INVALID_ARG, "null graph");
    const hipError_t he = hipGraphLaunch(exec, stream);
    return he == hipSuccess ? XCORR_OK : hip_fail((int)he, "graph launch");
}

void xcorr_graph_destroy(hipGraphExec_t exec)
{
    if (exec) (void)hipGraphExecDestroy(exec);
}

}  // extern "C"

// ------------------------------------------------------------------ F-engine

struct xcorr_fengine {
    int nstation = 0, npol = 0, nchan = 0, nframes = 0, nin = 0;
    float gain = 1.0f;
    int device = 0;
};

extern "C" {

xcorr_fengine_t *xcorr_fengine_create(int nstation, int npol, int nchan, int nframes, float gain)
{
    if (nstation < 1 || (npol != 1 && npol != 2) || nframes < 0) {
        fail(XCORR_ERR_INVALID_ARG, "need nstation >= 1, npol in {1, 2}, nframes >= 0");
        return nullptr;
    }
    if (nchan < 64 || nchan > 2048 || (nchan & (nchan - 1))) {
        fail(XCORR_ERR_INVALID_ARG, "nchan (the transform length) must be a power of two in 64..2048");
        return nullptr;
    }
    if (!(gain > 0.0f) || gain > 1e30f) {
        fail(XCORR_ERR_INVALID_ARG, "gain must be a positive finite number");
        return nullptr;
    }
    const int64_t nin = (int64_t)nstation * npol;
    if (nin > 65536 || (int64_t)nframes * nchan * nin > ((int64_t)1 << 40)) {
        fail(XCORR_ERR_RANGE, "too many inputs or samples");
        return nullptr;
    }
    int dev = 0;
    const hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) {
        hip_fail((int)he, "hipGetDevice");
        return nullptr;
    }
    xcorr_fengine *e = new (std::nothrow) xcorr_fengine;
    if (!e) {
        fail(XCORR_ERR_OOM, "host allocation");
        return nullptr;
    }
    e->nstation = nstation;
    e->npol = npol;
    e->nchan = nchan;
    e->nframes = nframes;
    e->nin = (int)nin;
    e->gain = gain;
    e->device = dev;
    return e;
}

size_t xcorr_fengine_in_bytes(const xcorr_fengine_t *e)
{
    return e ? (size_t)e->nin * e->nframes * e->nchan * 2 : 0;
}

size_t xcorr_fengine_out_bytes(const xcorr_fengine_t *e, int spectra)
{
    return e ? (size_t)e->nframes * e->nchan * e->nin * (spectra ? 8 : 2) : 0;
}

static int fengine_run(xcorr_fengine_t *e, const void *in, void *out, hipStream_t stream, bool spectra)
{
    if (!e) return fail(XCORR_ERR_INVALID_ARG, "null F-engine");
    if (e->nframes == 0) return XCORR_OK;
    if (!in || !out) return fail(XCORR_ERR_INVALID_ARG, "null input or output");
    if ((uintptr_t)in % 4 != 0) return fail(XCORR_ERR_INVALID_ARG, "the input must be 4-byte aligned");
    if (int rc = check_device(e->device)) return rc;
    const int rc = launch_fengine(in, out, e->nin, e->nchan, (int64_t)e->nframes * e->nchan, e->nframes, e->gain,
                                  spectra, stream);
    return rc ? hip_fail(rc, "F-engine launch") : XCORR_OK;
}

int xcorr_fengine_run(xcorr_fengine_t *e, const void *in, void *out, hipStream_t stream)
{
    return fengine_run(e, in, out, stream, false);
}

int xcorr_fengine_run_spectra(xcorr_fengine_t *e, const void *in, void *out, hipStream_t stream)
{
    return fengine_run(e, in, out, stream, true);
}

void xcorr_fengine_destroy(xcorr_fengine_t *e) { delete e; }

}  // extern "C"
