/*
 * xcorr.h -- C ABI of the MI355X X-engine.
 *
 * The X-engine of an FX correlator (Clark, La Plante and Greenhill, Sec. 2.1): for every
 * frequency channel f it integrates over time the outer product of the vector of station
 * signals with itself (Eq. 4), keeping only the lower triangle of the Hermitian result
 * (the Hermitian restriction stated after Eq. 4), with both polarisations of every station
 * in the vector:
 *
 *   V[f][s1*(s1+1)/2 + s2][p*npol + q] = sum_t x[t][f][s1][p] * conj(x[t][f][s2][q]),
 *   for 0 <= s2 <= s1 < nstation, 0 <= p, q < npol.
 *
 * Both cross-polarisation slots of an autocorrelation (s1 == s2, p != q) are stored; the
 * slot with p < q equals the conjugate of the slot with p > q.
 *
 * Layouts (all row-major, no padding):
 *   input   x[ntime][nchan][nstation][npol] complex samples, the corner-turned order of
 *           Sec. 4.1 (station fastest, then channel, then time);
 *   output  V[nchan][nstation*(nstation+1)/2][npol*npol] complex values, interleaved
 *           (real, imaginary), the packed correlation matrix of Algorithm 1 (Sec. 5).
 *
 * Sample formats (xcorr_in_dtype):
 *   XCORR_IN_CI8   2 bytes per sample: int8 real, int8 imaginary.
 *   XCORR_IN_CI4   1 byte per sample: real part in the high nibble, imaginary part in the
 *                  low nibble, each a two's complement integer in [-8, 7].
 *   XCORR_IN_CF32  8 bytes per sample: float real, float imaginary (F32_CMAC only).
 *   Integer samples are used as raw integers (no normalisation), so integer visibilities
 *   are exact integers.
 *
 * Arithmetic paths (xcorr_acc_dtype):
 *   XCORR_ACC_F32_CMAC        the paper's method: FP32 complex multiply-accumulate on the
 *                             vector ALUs (Sec. 4), 8 flops per complex MAC (Eq. 5).
 *   XCORR_ACC_I8_MMA_I32      int8 matrix cores, int32 accumulation.  CI8 samples must lie
 *                             in [-127, 127] (the conjugate side negates one operand).
 *   XCORR_ACC_F16_MMA_F32     fp16 matrix cores, fp32 accumulation (exact: |sample| <= 2048).
 *   XCORR_ACC_F8E4M3_MMA_F32  fp8 e4m3 matrix cores, fp32 accumulation; exact only for
 *                             |sample| <= 16, so it accepts CI4, or CI8 after
 *                             xcorr_set_max_abs(h, m) with m <= 16; otherwise the run is
 *                             refused with XCORR_ERR_UNSUPPORTED.
 *   XCORR_ACC_F32_MMA_F32     the plain path's FP32 arithmetic on the fp32 matrix cores
 *                             (v_mfma_f32_32x32x2_f32), fp32 accumulation; CI8 and CI4
 *                             samples (exact like the fp16 path), tiled kernel only.
 *   XCORR_ACC_F6E3M2_MMA_F32  fp6 e3m2 operands on the scaled f8f6f4 matrix cores, fp32
 *                             accumulation; e3m2 holds every integer of [-8, 8] exactly
 *                             (Sec. 2.3's few-bit digitised data), so it accepts CI4, or
 *                             CI8 after xcorr_set_max_abs(h, m) with m <= 8; otherwise the
 *                             run is refused with XCORR_ERR_UNSUPPORTED.  Tiled kernel, or
 *                             for CI4 the super-tiles (tile 512, after a pre-pass that
 *                             packs every 32-sample block of each input once).
 *
 * Exactness and the output type.  Integer samples with |component| <= max_abs grow any
 * accumulator by at most 2*max_abs^2 per sample.  The library integrates in windows of at
 * most floor((2^31-1) / (2*max_abs^2)) samples for int32 accumulators and
 * floor(2^24 / (2*max_abs^2)) samples for fp32 accumulators (below 2^24 every fp32 partial
 * sum of integers is exact, in any order); the wider accumulators of Sec. 2.3 then hold the
 * total.  A run of one window writes ci32 (int32 accumulators) or c64 (fp32 accumulators);
 * a run of several windows sums the windows on the GPU into ci64 or c128.  max_abs defaults
 * to 127 for CI8 on the int8 path, 128 for CI8 on the other paths and 8 for CI4;
 * xcorr_set_max_abs declares a smaller bound on the data (a promise by the caller, not
 * checked).  CF32 input runs one window and writes c64 unless xcorr_set_window asks for
 * shorter windows.
 *
 * Ownership and ordering.  Input and output are device pointers owned by the caller and
 * must stay valid until the work enqueued on `stream` has completed.  Every run is
 * asynchronous and stream ordered; the library never synchronises the host.  xcorr_run
 * overwrites the output with the visibilities of its ntime samples.  A handle owns its
 * device workspace and must not run on two streams at once.
 *
 * Errors.  Functions returning int give XCORR_OK (0) or a negative code below;
 * constructors return NULL.  xcorr_last_error() describes the last failure of the calling
 * thread.  Destroying NULL is a no-op.
 */
#ifndef XCORR_H
#define XCORR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    XCORR_IN_CI8 = 0,
    XCORR_IN_CI4 = 1,
    XCORR_IN_CF32 = 2
} xcorr_in_dtype;

typedef enum {
    XCORR_ACC_F32_CMAC = 0,
    XCORR_ACC_I8_MMA_I32 = 1,
    XCORR_ACC_F16_MMA_F32 = 2,
    XCORR_ACC_F8E4M3_MMA_F32 = 3,
    XCORR_ACC_F32_MMA_F32 = 4,
    XCORR_ACC_F6E3M2_MMA_F32 = 5
} xcorr_acc_dtype;

typedef enum {
    XCORR_OUT_CI32 = 0, /* int32 real, int32 imaginary */
    XCORR_OUT_CI64 = 1, /* int64 real, int64 imaginary */
    XCORR_OUT_C64 = 2,  /* float real, float imaginary */
    XCORR_OUT_C128 = 3  /* double real, double imaginary */
} xcorr_out_dtype;

enum {
    XCORR_OK = 0,
    XCORR_ERR_INVALID_ARG = -1, /* bad size, pointer or enumerator */
    XCORR_ERR_UNSUPPORTED = -2, /* combination that would not be exact */
    XCORR_ERR_OOM = -3,         /* device or host allocation failed */
    XCORR_ERR_HIP = -4,         /* a HIP runtime call failed (see xcorr_last_error) */
    XCORR_ERR_RANGE = -5        /* a size exceeds what the library indexes, or (with
                                   validation on) a sample component is outside the declared
                                   range */
};

/* ------------------------------------------------------------------ one correlation job */

typedef struct xcorr_handle xcorr_handle_t;

/*
 * Plan a job of nstation stations x npol (1 or 2) polarisations, nchan channels and ntime
 * samples (the sizes of Eq. 4 and Algorithm 1) on the current device.  Allocates no device
 * memory.  Returns NULL on error.
 */
xcorr_handle_t *xcorr_create(int nstation, int npol, int nchan, int ntime,
                             xcorr_in_dtype in_dtype, xcorr_acc_dtype acc_dtype);

/* Declare that every real and imaginary component satisfies |v| <= max_abs (1..127 for
 * CI8, 1..8 for CI4).  Re-plans the accumulation windows and may change the output type. */
int xcorr_set_max_abs(xcorr_handle_t *h, int max_abs);

/* Choose the kernel shape (Sec. 4.2's tiling of the triangle, re-planned for gfx950):
 *   0    automatic (the default): 512 when allowed and its padded last super-row costs at
 *        most 15 % more computed blocks than 128-tiles, else 256 when allowed and
 *        nin > 192, else 128 (64 when nin <= 64; always 64 for F32_CMAC);
 *   64, 128  square tiles of that many inputs, one workgroup per (channel, tile, window);
 *   256  whole channel: one persistent workgroup per compute unit holds the triangle of a
 *        channel and reads every sample once; needs CI8 input, the int8 or fp16 path and
 *        nin <= 256, a multiple of 8.  An input pointer that is not 16-byte aligned runs
 *        128-tiles instead;
 *   512  super-tiles: the triangle of each channel cut into 256-input triangles and
 *        256 x 128 rectangles, each held by one persistent workgroup (two launches); needs
 *        CI4 input on the int8, fp8 or fp6 path, or CI8 input on the int8 path, and nin a
 *        multiple of 16 in 272..2048; for CI4 on the int8 path also windows of at most
 *        (2^31 - 1) / (256 max_abs^2) samples (its operands are the samples times 8, or 16
 *        on the row side of a rectangle); on the fp6 path windows of a multiple of 32
 *        samples (or one window), and a workspace the handle allocates on its first run
 *        or autotune with this shape (48 bytes per input, padded to a multiple of 256
 *        inputs, per 32-sample block per channel: 1.5 x the input bytes plus the padding;
 *        held until xcorr_destroy; the first run must not be inside a graph capture, else
 *        XCORR_ERR_UNSUPPORTED; XCORR_ERR_OOM if it cannot be allocated).  The batch and
 *        stream entry points have no such workspace and run fp6 jobs on 128-tiles.
 *        Same alignment fallback.
 * All shapes give bit-identical visibilities.  XCORR_ERR_INVALID_ARG for a shape the job
 * does not allow (the handle keeps its previous shape).  Resets the kernel variant to 0 and
 * keeps the staging (tiles 256 / 512 need XCORR_STAGE_LDS). */
int xcorr_set_tile(xcorr_handle_t *h, int tile);

/* The kernel shape the handle runs (64, 128, 256 or 512), or an error code. */
int xcorr_get_tile(const xcorr_handle_t *h);

/* Operand staging of the tiled kernel (tiles 64 / 128): the software-managed cache of
 * Sec. 4.4 (operands staged in LDS, the default) or the hardware-managed cache of Sec. 4.3
 * (every wave loads its own operands from memory through the L1 and L2 caches, no LDS).
 * The whole-channel and super-tiled kernels always stage in LDS, so XCORR_STAGE_CACHE
 * switches such a handle to the automatic tiled shape (128, or 64 for nin <= 64).  Not for
 * the FP32 CMAC path (XCORR_ERR_UNSUPPORTED).  Same visibilities either way. */
typedef enum { XCORR_STAGE_LDS = 0, XCORR_STAGE_CACHE = 1 } xcorr_staging;
int xcorr_set_staging(xcorr_handle_t *h, int staging);
int xcorr_get_staging(const xcorr_handle_t *h);

/* Compile-time variant of the kernel (the tuning parameters of Sec. 4.3 / 4.4 fixed per
 * kernel build): whole-channel kernel (tile 256) 0..3, fp16 0..7 — bit 0 keeps one time
 * block fewer in the LDS copy ring (int8: 3 instead of 4 blocks of 64 samples; fp16: 4
 * instead of 5 of 32), bit 1 swaps which of the two waves sharing a SIMD takes the
 * five-block work list, bit 2 (fp16) converts each block to fp16 on all eight waves
 * instead of the four five-block waves;
 * super-tiles (tile 512) 0..3 — bit 0 uses a three-block instead of a four-block ring, bit 1
 * stages the rectangles' column operands also in rotated (-im, re) form, so that no wave
 * rotates a fragment (fp6 super-tiles: 0..1 — variant 0 reads the rotated row fragments
 * from LDS, variant 1 exchanges the lane halves of the plain ones in registers); the other
 * kernels have variant 0 only.  XCORR_ERR_INVALID_ARG outside that range.  Same
 * visibilities for every variant. */
int xcorr_set_variant(xcorr_handle_t *h, int variant);
int xcorr_get_variant(const xcorr_handle_t *h);

/* Accumulation window (the dump interval of Sec. 2.3's wider accumulators): integrate in
 * windows of `window` samples, each summed into the wide output (ci64 / c128) when the run
 * has more than one.  0 (the default) takes the longest exact window (see the exactness
 * note above); a positive value must not exceed xcorr_window_limit for the handle's
 * format, path and max_abs (XCORR_ERR_UNSUPPORTED otherwise: the sums would not be exact).
 * Shorter windows give the same visibilities; they only add window sums.  A later
 * xcorr_set_max_abs keeps the requested window.  XCORR_ERR_INVALID_ARG for window < 0. */
int xcorr_set_window(xcorr_handle_t *h, int window);

/* Autotuner (the parameter search of Sec. 4.3 / 4.4 and 6, done on the device): run every
 * kernel shape the job allows — tile (xcorr_set_tile) x staging (xcorr_set_staging) x
 * kernel variant (xcorr_set_variant) — `reps` times (after one warm-up; before the first
 * shape, `reps` untimed runs bring the clocks up) on `in` / `out` on `stream`, timed with
 * HIP events, keep the fastest on the handle and record it in the
 * process-wide tuning cache under the job's class: the current device's architecture
 * (e.g. "gfx950"), nstation, npol, formats, max_abs, requested window, and the power-of-two
 * buckets ceil(log2(nchan)) and ceil(log2(ntime)).  Handles created or re-planned later
 * whose job falls in a cached class start with the tuned shape.  Returns the chosen tile
 * (> 0) or an error code.  Synchronises the host with `stream`; `out` holds the
 * visibilities of `in` afterwards (every shape gives the same bits).  reps in 1..1000. */
int xcorr_autotune(xcorr_handle_t *h, const void *in, void *out, hipStream_t stream, int reps);

/* The shapes the handle's last xcorr_autotune timed: returns their number; for 0 <= k <
 * that number, fills the k-th shape and its mean time per run in microseconds (null
 * pointers are skipped). */
int xcorr_autotune_results(const xcorr_handle_t *h, int k, int *tile, int *staging, int *variant, double *us);

/* Kernel shape cached for a job's class on architecture `arch` (NULL: the current
 * device's; max_abs 0: the default bound): the tile, with *staging and *variant filled
 * (when not NULL); 0 if none; or an error code. */
int xcorr_autotune_lookup(const char *arch, int nstation, int npol, int nchan, int ntime, xcorr_in_dtype in_dtype,
                          xcorr_acc_dtype acc_dtype, int max_abs, int *staging, int *variant);

/* Keep the tuning cache in a text file (one JSON object per line: "arch", the class,
 * "tile", "staging", "variant" and the measured "us"); load merges into the cache.  Return
 * the number of entries, or XCORR_ERR_INVALID_ARG on an I/O or format error. */
int xcorr_autotune_save(const char *path);
int xcorr_autotune_load(const char *path);
void xcorr_autotune_clear(void);

/* Compute the visibilities of `in` (device, xcorr_in_bytes) into `out` (device,
 * xcorr_out_bytes) on `stream` (0 = the null stream).  The device the handle was created on
 * must be current (XCORR_ERR_INVALID_ARG otherwise). */
int xcorr_run(xcorr_handle_t *h, const void *in, void *out, hipStream_t stream);

/* Range check of integer samples (the exactness conditions of Sec. 2.3: every window and
 * every operand type is sized for components bounded by max_abs; on the int8 path a
 * component of -128 would overflow when the imaginary product negates it).  Counts the
 * real and imaginary components of `in` (device, xcorr_in_bytes bytes, any alignment)
 * outside [-max_abs, max_abs] (the declared bound, else the format's default: 127 for CI8 on
 * the int8 path, so -128 counts) and writes the count to *nbad (host).  One pass over the
 * input on `stream`, then waits for the stream: not allowed while the stream is capturing a
 * graph (XCORR_ERR_UNSUPPORTED).  The first call allocates an 8-byte device counter, which
 * xcorr_destroy frees.  CF32 input: *nbad = 0. */
int xcorr_validate(xcorr_handle_t *h, const void *in, hipStream_t stream, int64_t *nbad);

/* on = 1: every xcorr_run first runs xcorr_validate and, if any component is out of range,
 * returns XCORR_ERR_RANGE without computing (out untouched); such runs wait for the stream
 * and cannot be captured.  on = 0 (the default): no check. */
int xcorr_set_validation(xcorr_handle_t *h, int on);

void xcorr_destroy(xcorr_handle_t *h);

size_t xcorr_in_bytes(const xcorr_handle_t *h);
size_t xcorr_out_bytes(const xcorr_handle_t *h);
int xcorr_out_type(const xcorr_handle_t *h); /* an xcorr_out_dtype, or < 0 on error */

/* Text of the last error on the calling thread ("" if none). */
const char *xcorr_last_error(void);

/* ------------------------------------------------------------------ batches of jobs */

/*
 * Many independent jobs of different sizes (uneven sub-arrays, channel counts and
 * integration lengths) in one persistent launch.  The increase of thread blocks with the
 * number of channels is what keeps the GPU busy at small N (Sec. 6.1); a batch gets the
 * same effect from many small jobs.  All jobs share the sample format and the arithmetic
 * path; each job has its own input and output buffers with the layouts above.
 */
typedef struct {
    int nstation;
    int npol;
    int nchan;
    int ntime;
} xcorr_job;

typedef struct xcorr_batch xcorr_batch_t;

/* Plan njobs jobs; uploads the work list (one item per job, channel, tile and window) to
 * the current device.  Returns NULL on error. */
xcorr_batch_t *xcorr_batch_create(int njobs, const xcorr_job *jobs, xcorr_in_dtype in_dtype,
                                  xcorr_acc_dtype acc_dtype);

/* Component bound for every job (as xcorr_set_max_abs); rebuilds the work list. */
int xcorr_batch_set_max_abs(xcorr_batch_t *b, int max_abs);

/* in[j], out[j]: device buffers of job j (host arrays of njobs device pointers).  Enqueues
 * on `stream`: a small upload of the job table, zero fills of the outputs that sum several
 * windows, the launches of each job that the planner gives the whole-channel or the
 * super-tiled kernel (see xcorr_set_tile), and one persistent launch of the tiled kernel
 * over the work items of all other jobs.  May wait on the host for the previous run's table
 * upload to finish.  The device the batch was created on must be current. */
int xcorr_batch_run(xcorr_batch_t *b, const void *const *in, void *const *out, hipStream_t stream);

size_t xcorr_batch_in_bytes(const xcorr_batch_t *b, int job);
size_t xcorr_batch_out_bytes(const xcorr_batch_t *b, int job);
int xcorr_batch_out_type(const xcorr_batch_t *b, int job);
/* Work items of the persistent tiled launch (jobs on the whole-channel or super-tiled
 * kernels excluded). */
int64_t xcorr_batch_items(const xcorr_batch_t *b);
void xcorr_batch_destroy(xcorr_batch_t *b);

/* For callers that cannot allocate memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the work of xcorr_batch_create(njobs, jobs,
 * in_dtype, acc_dtype) + xcorr_batch_set_max_abs(max_abs) (max_abs 0: the format's default;
 * 8-bit samples on the fp8 path need 1..16) + xcorr_batch_run(in, out, stream), in one
 * call that allocates nothing on the host or the device and gives the same visibilities.
 * The jobs that run on the tiled kernel take their work from a fixed workspace inside the
 * library instead of allocated buffers: a job table, queue counters and the generated
 * work list's counts, XCORR_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on a
 * GPU until the process ends.  The job table reaches it by kernel arguments and the
 * counters are cleared on `stream` at every call, so the call only enqueues work and
 * returns (nothing is read from host memory afterwards).  Every call on a GPU shares that
 * GPU's workspace: calls that overlap on one GPU (on different streams, or from several
 * threads without ordering) race and give wrong results; calls ordered on one stream are
 * safe.  XCORR_ERR_INVALID_ARG for njobs outside 1..XCORR_NOALLOC_MAX_JOBS, null arrays or
 * pointers, or a bad max_abs; otherwise the errors of create / set_max_abs / run. */
#define XCORR_NOALLOC_MAX_JOBS 256
#define XCORR_NOALLOC_SCRATCH_BYTES 43520
int xcorr_batch_run_noalloc(int njobs, const xcorr_job *jobs, xcorr_in_dtype in_dtype, xcorr_acc_dtype acc_dtype,
                            int max_abs, const void *const *in, void *const *out, hipStream_t stream);

/* ------------------------------------------------------------------ streaming integration */

/*
 * The integrated X-engine of Algorithm 1 (Sec. 5): the input of a long integration arrives
 * from the host in chunks of chunk_ntime samples; chunk p+1 is copied to the device while
 * chunk p is correlated, and every chunk's visibilities are added to running totals on the
 * device.  The totals are always wide (ci64 for the int8 path, c128 otherwise) and exact:
 * each chunk is integrated in exact windows (see above) and added to the totals in
 * int64 / fp64.
 *
 * The stream owns a copy stream (default priority), two device chunk buffers and their
 * events.  Host chunks should be pinned (hipHostMalloc) for the copies to be asynchronous.
 * Release point: a chunk passed to push p may be changed or freed by the caller once push
 * p + 2 has returned (push p + 2 waits on the host for the copy of chunk p to finish, as
 * Algorithm 1 synchronises each iteration), or once xcorr_stream_end has been called and
 * `stream` synchronised.  Pushes recorded by xcorr_stream_capture do not wait.
 *
 * Differences from a create(total_ntime, dump_every) / push / finish interface: the
 * integration length is the number of pushes between begin and end (any number), and the
 * int32 / fp32 accumulators are dumped into the wide totals at the end of every chunk and,
 * within a chunk, every xcorr_stream_set_window samples (default: the longest exact
 * window).
 */
typedef struct xcorr_stream xcorr_stream_t;

xcorr_stream_t *xcorr_stream_create(int nstation, int npol, int nchan, int chunk_ntime,
                                    xcorr_in_dtype in_dtype, xcorr_acc_dtype acc_dtype);

/* As xcorr_set_max_abs, for every chunk; call before xcorr_stream_begin. */
int xcorr_stream_set_max_abs(xcorr_stream_t *s, int max_abs);

/* As xcorr_set_window, within every chunk (dumps also happen at every chunk end); call
 * before xcorr_stream_begin. */
int xcorr_stream_set_window(xcorr_stream_t *s, int window);

/* Start an integration into `out` (device, xcorr_stream_out_bytes, type
 * xcorr_stream_out_type): zero it on `stream`. */
int xcorr_stream_begin(xcorr_stream_t *s, void *out, hipStream_t stream);

/* Copy one chunk (host, xcorr_stream_chunk_bytes, layout [chunk_ntime][nchan][nstation][npol])
 * to the device and add its visibilities to the totals; both steps are enqueued, ordered
 * after earlier work on `stream`. */
int xcorr_stream_push(xcorr_stream_t *s, const void *host_chunk, hipStream_t stream);

/* Finish the integration: all of its work is ordered before later work on `stream`.
 * Returns the number of samples integrated (>= 0) or an error code. */
int64_t xcorr_stream_end(xcorr_stream_t *s, hipStream_t stream);

size_t xcorr_stream_chunk_bytes(const xcorr_stream_t *s);
size_t xcorr_stream_out_bytes(const xcorr_stream_t *s);
int xcorr_stream_out_type(const xcorr_stream_t *s);
void xcorr_stream_destroy(xcorr_stream_t *s);

/* Record a whole integration of nchunk chunks (begin, one push per host_chunks[c], end)
 * into a HIP graph, once, and return it instantiated in *exec.  Every launch of the graph
 * (xcorr_graph_launch, or hipGraphLaunch) zeroes `out` and integrates the chunks as they
 * are in host memory at that time, with the same copy/compute overlap; the host pointers
 * and `out` are baked in and must stay valid while the graph is used.  Launches of one
 * graph, and runs of its stream object, must not overlap.  Nothing is enqueued by the
 * capture itself.  On failure *exec is NULL and an error code is returned. */
int xcorr_stream_capture(xcorr_stream_t *s, int nchunk, const void *const *host_chunks, void *out,
                         hipGraphExec_t *exec);
int xcorr_graph_launch(hipGraphExec_t exec, hipStream_t stream);
void xcorr_graph_destroy(hipGraphExec_t exec);

/* ------------------------------------------------------------------ host-only planning */

/*
 * What a plan does, without touching a GPU.  The useful work is the Eq. 5 count
 * (one complex MAC per input pair of the lower triangle including autocorrelations, per
 * channel and sample); the computed work adds the pairs that tiles on the diagonal and the
 * zero padding of the last tile compute without storing (the wasted work of Sec. 6.1).
 */
typedef struct {
    int nin;             /* nstation * npol */
    int tile;            /* inputs per side of a square tile; 256: whole channel */
    int ntile_side;      /* ceil(nin / tile) */
    int tiles_per_chan;  /* ntile_side * (ntile_side + 1) / 2 */
    int window;          /* samples per accumulation window */
    int nwindows;        /* ceil(ntime / window) */
    int max_abs;         /* component bound the windows assume */
    int out_dtype;       /* xcorr_out_dtype */
    int64_t nitems;      /* work items (channel, tile, window) */
    int64_t useful_cmacs;   /* nin*(nin+1)/2 * nchan * ntime */
    int64_t computed_cmacs; /* complex MACs the kernels execute */
    size_t in_bytes;
    size_t out_bytes;
} xcorr_plan_info;

/* Plan a job as xcorr_create + xcorr_set_max_abs (max_abs 0: the default) +
 * xcorr_set_tile (tile 0: automatic) + xcorr_set_window (window 0: longest exact) would. */
int xcorr_plan(int nstation, int npol, int nchan, int ntime, xcorr_in_dtype in_dtype,
               xcorr_acc_dtype acc_dtype, int max_abs, int tile, int window, xcorr_plan_info *info);

/* Largest window (samples) for which the accumulators of acc_dtype stay exact with
 * components bounded by max_abs; < 0 on a bad argument. */
int64_t xcorr_window_limit(xcorr_in_dtype in_dtype, xcorr_acc_dtype acc_dtype, int max_abs);

/* Inverse of the triangular tile numbering g = by*(by+1)/2 + bx, 0 <= bx <= by
 * (Sec. 4.2), in exact integer arithmetic.  Returns XCORR_ERR_INVALID_ARG for g < 0. */
int xcorr_tile_coords(int64_t g, int64_t *bx, int64_t *by);

/* ------------------------------------------------------------------ F-engine and corner turn */

/*
 * The F-engine of the FX correlator (Sec. 2.1): every input's digitised complex signal is
 * Fourier transformed nchan samples at a time, one nchan-point DFT per input every nchan
 * samples, and the corner turn reorders the spectra from station-major to the
 * channel-major order the X-engine reads (Sec. 4.1).  Output channel k of frame t is DFT bin
 * k of samples t nchan .. t nchan + nchan - 1, X[k] = sum_n x[n] exp(-2 pi i k n / nchan)
 * (natural order, no window or filter bank), times `gain`, requantised to XCORR_IN_CI8
 * samples: each component rounded half away from zero and clipped to [-127, 127], so the
 * output can go straight to any X-engine path.
 *
 * Layouts:
 *   input   x[nin][nframes * nchan] complex int8 (re, im), nin = nstation * npol (input
 *           station * npol + pol), each input's samples contiguous; 4-byte aligned;
 *   output  [nframes][nchan][nin] complex int8 (re, im): xcorr_create(nstation, npol,
 *           nchan, nframes, XCORR_IN_CI8, ...) reads it as is;
 *   spectra (xcorr_fengine_run_spectra) the same order as complex float (re, im), gain
 *           applied, not rounded.
 * nchan a power of two in 64..2048; gain > 0.  Device pointers owned by the caller; runs are
 * asynchronous on `stream`; the current device must be the one the object was created on.
 * Computed in fp32: a value within a few fp32 rounding errors of a rounding boundary may
 * land on either neighbouring integer.
 */
typedef struct xcorr_fengine xcorr_fengine_t;

xcorr_fengine_t *xcorr_fengine_create(int nstation, int npol, int nchan, int nframes, float gain);
size_t xcorr_fengine_in_bytes(const xcorr_fengine_t *e);
size_t xcorr_fengine_out_bytes(const xcorr_fengine_t *e, int spectra);
int xcorr_fengine_run(xcorr_fengine_t *e, const void *in, void *out, hipStream_t stream);
int xcorr_fengine_run_spectra(xcorr_fengine_t *e, const void *in, void *out, hipStream_t stream);
void xcorr_fengine_destroy(xcorr_fengine_t *e);

#ifdef __cplusplus
}
#endif

#endif /* XCORR_H */
