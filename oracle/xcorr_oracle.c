/*
 * CPU oracle for the X-engine.  TEST INFRASTRUCTURE: only the tests, the smoke check and
 * the benchmark's CPU-baseline leg may load or call this file's library.  It shares no code
 * with the GPU path.
 *
 * What it computes (Sec. 2.1, Eq. 4, with the Hermitian restriction to the lower triangle
 * stated right after it, and dual polarisation doubling the input vector):
 *
 *   out[f][s1*(s1+1)/2 + s2][p*npol + q] = sum_{t=0}^{ntime-1} x[t][f][s1][p] * conj(x[t][f][s2][q])
 *
 * for every channel f, every station pair s1 >= s2 and every polarisation pair (p, q),
 * including both cross-polarisation slots of an autocorrelation (s1 == s2).
 *
 * Input layout is the corner-turned order of Sec. 4.1: station*pol fastest, then channel,
 * then time.  Output is the packed triangle of Algorithm 1 (Sec. 5), one npol x npol block
 * of complex values per station baseline, stored as interleaved (real, imaginary).
 *
 * Integer samples accumulate in int64 and float samples in double: every value of every
 * workload used here is an exact integer far below 2^53, so the result is exact.
 *
 * The loops follow the definition literally: channel, then baseline, then polarisation
 * pair, then the sum over time.  The only parallelism is over channels.
 */
#include <stddef.h>
#include <stdint.h>

/* Sample formats (see the public header of the library for the same contract). */
enum { ORACLE_CI8 = 0, ORACLE_CI4 = 1, ORACLE_CF32 = 2 };

/* One complex sample of input `n` (flat index over [t][f][input]). */
static void sample_int(const void *x, int fmt, size_t n, int64_t *re, int64_t *im)
{
    if (fmt == ORACLE_CI8) {
        const int8_t *p = (const int8_t *)x;
        *re = p[2 * n];
        *im = p[2 * n + 1];
    } else {
        /* 4-bit complex: real part in the high nibble, imaginary part in the low nibble,
         * each a two's complement number in [-8, 7]. */
        const uint8_t *p = (const uint8_t *)x;
        int r = (p[n] >> 4) & 0xF;
        int i = p[n] & 0xF;
        *re = r >= 8 ? r - 16 : r;
        *im = i >= 8 ? i - 16 : i;
    }
}

static size_t tri(size_t s1, size_t s2) { return s1 * (s1 + 1) / 2 + s2; }

/*
 * Integer samples.  chans[0..nsel) lists the channels to compute (each in [0, nchan));
 * out has nsel * nstation*(nstation+1)/2 * npol*npol * 2 int64 entries.
 * Returns 0, or -1 on a bad argument.
 */
int oracle_xcorr_int(const void *x, int fmt, int nstation, int npol, int nchan, int ntime,
                     const int *chans, int nsel, int64_t *out)
{
    if (!x || !out || !chans || nstation < 1 || npol < 1 || nchan < 1 || ntime < 0 || nsel < 0)
        return -1;
    if (fmt != ORACLE_CI8 && fmt != ORACLE_CI4)
        return -1;
    const size_t nin = (size_t)nstation * npol;
    const size_t nbl = tri(nstation, 0);
    const size_t npp = (size_t)npol * npol;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nsel; ++c) {
        const size_t f = (size_t)chans[c];
        for (size_t s1 = 0; s1 < (size_t)nstation; ++s1)
            for (size_t s2 = 0; s2 <= s1; ++s2)
                for (size_t p = 0; p < (size_t)npol; ++p)
                    for (size_t q = 0; q < (size_t)npol; ++q) {
                        int64_t acc_re = 0, acc_im = 0;
                        for (size_t t = 0; t < (size_t)ntime; ++t) {
                            const size_t row = (t * (size_t)nchan + f) * nin;
                            int64_t ar, ai, br, bi;
                            sample_int(x, fmt, row + s1 * npol + p, &ar, &ai);
                            sample_int(x, fmt, row + s2 * npol + q, &br, &bi);
                            /* (ar + i ai) * conj(br + i bi) */
                            acc_re += ar * br + ai * bi;
                            acc_im += ai * br - ar * bi;
                        }
                        int64_t *o = out + (((size_t)c * nbl + tri(s1, s2)) * npp + p * npol + q) * 2;
                        o[0] = acc_re;
                        o[1] = acc_im;
                    }
    }
    return 0;
}

/* Float samples (complex float32, interleaved), accumulated in double. */
int oracle_xcorr_f64(const float *x, int nstation, int npol, int nchan, int ntime,
                     const int *chans, int nsel, double *out)
{
    if (!x || !out || !chans || nstation < 1 || npol < 1 || nchan < 1 || ntime < 0 || nsel < 0)
        return -1;
    const size_t nin = (size_t)nstation * npol;
    const size_t nbl = tri(nstation, 0);
    const size_t npp = (size_t)npol * npol;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nsel; ++c) {
        const size_t f = (size_t)chans[c];
        for (size_t s1 = 0; s1 < (size_t)nstation; ++s1)
            for (size_t s2 = 0; s2 <= s1; ++s2)
                for (size_t p = 0; p < (size_t)npol; ++p)
                    for (size_t q = 0; q < (size_t)npol; ++q) {
                        double acc_re = 0.0, acc_im = 0.0;
                        for (size_t t = 0; t < (size_t)ntime; ++t) {
                            const size_t row = (t * (size_t)nchan + f) * nin;
                            const float *a = x + 2 * (row + s1 * npol + p);
                            const float *b = x + 2 * (row + s2 * npol + q);
                            acc_re += (double)a[0] * b[0] + (double)a[1] * b[1];
                            acc_im += (double)a[1] * b[0] - (double)a[0] * b[1];
                        }
                        double *o = out + (((size_t)c * nbl + tri(s1, s2)) * npp + p * npol + q) * 2;
                        o[0] = acc_re;
                        o[1] = acc_im;
                    }
    }
    return 0;
}

/* Number of threads the OpenMP runtime will use (reported beside timings). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
