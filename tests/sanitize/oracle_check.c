/*
 * The X-engine oracle's C library run under AddressSanitizer and
 * UndefinedBehaviorSanitizer on small seeded inputs of every sample format, with the
 * argument checks and the edge shapes (no samples, no channels selected, one station, one
 * polarisation, a channel subset).  Each result is compared with a second evaluation of
 * Eq. 4 in another loop order (time outermost, every pair updated per sample), so that
 * the run also checks the values.  Prints "ok" and exits 0 when everything holds.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_xcorr_int(const void *x, int fmt, int nstation, int npol, int nchan, int ntime,
                     const int *chans, int nsel, int64_t *out);
int oracle_xcorr_f64(const float *x, int nstation, int npol, int nchan, int ntime,
                     const int *chans, int nsel, double *out);

static uint64_t g_state = 0x9E3779B97F4A7C15ULL;
static uint64_t next_u64(void)
{
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return g_state * 0x2545F4914F6CDD1DULL;
}

static int g_fail = 0;
static void check(int ok, const char *what, int a)
{
    if (!ok && g_fail++ < 20) fprintf(stderr, "FAIL %s (%d)\n", what, a);
}

/* component value of input n (flat over [t][f][input]) in the second evaluation */
static void comp(const void *x, int fmt, size_t n, double *re, double *im)
{
    if (fmt == 0) {
        const int8_t *p = (const int8_t *)x;
        *re = p[2 * n];
        *im = p[2 * n + 1];
    } else if (fmt == 1) {
        const uint8_t b = ((const uint8_t *)x)[n];
        const int hi = b >> 4, lo = b & 15;
        *re = hi - ((hi & 8) ? 16 : 0);
        *im = lo - ((lo & 8) ? 16 : 0);
    } else {
        const float *p = (const float *)x;
        *re = p[2 * n];
        *im = p[2 * n + 1];
    }
}

static void run_case(int fmt, int ns, int np, int nc, int nt, int nsel)
{
    const size_t nin = (size_t)ns * np, nsamp = (size_t)nt * nc * nin;
    const size_t bps = fmt == 0 ? 2 : (fmt == 1 ? 1 : 8);
    unsigned char *x = malloc(nsamp * bps + 1);
    for (size_t i = 0; i < nsamp * bps; ++i) x[i] = (unsigned char)(next_u64() >> 56);
    if (fmt == 2)
        for (size_t i = 0; i < 2 * nsamp; ++i) ((float *)x)[i] = (float)((int)(next_u64() >> 58) - 32);
    int *chans = malloc(sizeof(int) * (nsel + 1));
    for (int c = 0; c < nsel; ++c) chans[c] = (int)((c * 7 + 3) % nc);
    const size_t nbl = (size_t)ns * (ns + 1) / 2, npp = (size_t)np * np;
    const size_t nout = (size_t)nsel * nbl * npp * 2;
    int64_t *oi = malloc(sizeof(int64_t) * (nout + 1));
    double *od = malloc(sizeof(double) * (nout + 1));
    double *want = calloc(nout + 1, sizeof(double));
    int rc = fmt == 2 ? oracle_xcorr_f64((const float *)x, ns, np, nc, nt, chans, nsel, od)
                      : oracle_xcorr_int(x, fmt, ns, np, nc, nt, chans, nsel, oi);
    check(rc == 0, "oracle accepted valid arguments", fmt);
    for (int t = 0; t < nt; ++t)
        for (int c = 0; c < nsel; ++c)
            for (size_t i = 0; i < nin; ++i)
                for (size_t j = 0; j <= i; ++j) {
                    const size_t s1 = i / np, p = i % np, s2 = j / np, q = j % np;
                    if (s2 > s1) continue;
                    const size_t row = ((size_t)t * nc + chans[c]) * nin;
                    double ar, ai, br, bi;
                    comp(x, fmt, row + i, &ar, &ai);
                    comp(x, fmt, row + j, &br, &bi);
                    /* baseline (s1, s2); when s1 == s2 both polarisation orders are kept */
                    double *w = want + (((size_t)c * nbl + s1 * (s1 + 1) / 2 + s2) * npp + p * np + q) * 2;
                    w[0] += ar * br + ai * bi;
                    w[1] += ai * br - ar * bi;
                    if (s1 == s2 && p != q) {
                        double *v = want + (((size_t)c * nbl + s1 * (s1 + 1) / 2 + s2) * npp + q * np + p) * 2;
                        v[0] += br * ar + bi * ai;
                        v[1] += bi * ar - br * ai;
                    }
                }
    for (size_t k = 0; k < nout; ++k) {
        const double got = fmt == 2 ? od[k] : (double)oi[k];
        check(got == want[k], "oracle value", (int)k);
    }
    free(x);
    free(chans);
    free(oi);
    free(od);
    free(want);
}

int main(void)
{
    static const int shapes[][5] = {
        /* nstation, npol, nchan, ntime, nsel */
        {1, 1, 1, 1, 1}, {1, 2, 3, 5, 3}, {5, 2, 3, 7, 3}, {7, 1, 4, 9, 2},
        {4, 2, 2, 0, 2}, {6, 2, 5, 3, 0},  {33, 2, 2, 17, 2}, {3, 2, 9, 4, 5},
    };
    for (int fmt = 0; fmt < 3; ++fmt)
        for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s)
            run_case(fmt, shapes[s][0], shapes[s][1], shapes[s][2], shapes[s][3], shapes[s][4]);
    /* argument checks: each call is refused before it reads anything */
    int8_t x[8] = {0};
    int ch = 0;
    int64_t o[8];
    double od[8];
    check(oracle_xcorr_int(NULL, 0, 1, 1, 1, 1, &ch, 1, o) == -1, "null input", 0);
    check(oracle_xcorr_int(x, 0, 0, 1, 1, 1, &ch, 1, o) == -1, "no stations", 0);
    check(oracle_xcorr_int(x, 2, 1, 1, 1, 1, &ch, 1, o) == -1, "float format on the integer entry", 0);
    check(oracle_xcorr_int(x, 0, 1, 1, 1, -1, &ch, 1, o) == -1, "negative ntime", 0);
    check(oracle_xcorr_f64(NULL, 1, 1, 1, 1, &ch, 1, od) == -1, "null float input", 0);
    check(oracle_xcorr_f64((const float *)x, 1, 0, 1, 1, &ch, 1, od) == -1, "no polarisations", 0);
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("ok\n");
    return 0;
}
