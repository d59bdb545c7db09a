// Host-side checks of the planner and the tune cache, built with AddressSanitizer and
// UndefinedBehaviorSanitizer (no GPU calls: these sources hold the library's host logic).
// Exits 0 and prints "ok" when every check holds; a sanitizer report aborts the run.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <string>

#include "plan.h"
#include "tune.h"
#include "xcorr.h"
#include "xeng.h"

using namespace xc;

namespace {

uint64_t g_state = 0x2545F4914F6CDD1DULL;
uint64_t next_u64()
{
    // xorshift64*: a fixed, reproducible stream of arguments
    g_state ^= g_state >> 12;
    g_state ^= g_state << 25;
    g_state ^= g_state >> 27;
    return g_state * 0x2545F4914F6CDD1DULL;
}
template <size_t N>
int pick(const int (&v)[N])
{
    return v[next_u64() % N];
}

int g_fail = 0;
void check(bool ok, const char *what, long long a = 0, long long b = 0)
{
    if (!ok && g_fail++ < 20) fprintf(stderr, "FAIL %s (%lld, %lld)\n", what, a, b);
}

void plans()
{
    static const int ns[] = {1, 2, 3, 4, 5, 7, 8, 17, 31, 32, 33, 64, 96, 97, 128, 129, 136, 200, 256, 300, 512, 1024, 0};
    static const int np[] = {1, 2, 2, 1, 2, 3};
    static const int nc[] = {1, 2, 3, 7, 64, 1024, 0};
    static const int nt[] = {0, 1, 2, 31, 63, 64, 65, 500, 520, 521, 4096, 66572, 66573, 1 << 20, 7, 100, -1};
    static const int fmt[] = {IN_CI8, IN_CI8, IN_CI4, IN_CI4, IN_CF32, 3};
    static const int acc[] = {ACC_F32_CMAC, ACC_I8, ACC_I8, ACC_F16, ACC_F16, ACC_F8, ACC_F32M, ACC_F6, 6};
    static const int mabs[] = {0, 0, 0, 0, 0, 1, 7, 8, 9, 16, 17, 18, 127, 128, 129};
    static const int tile[] = {0, 0, 0, 0, 0, 0, 64, 128, 256, 512, 100};
    static const int win[] = {0, 0, 0, 0, 0, 0, 1, 64, 520, 66572, 1 << 24, -5};
    static const int stg[] = {0, 0, 0, 0, 0, 1, 2};
    static const int var[] = {0, 0, 0, 0, 0, 1, 2, 3, 4};
    int nok = 0;
    for (int it = 0; it < 200000; ++it) {
        const int s = pick(ns), p = pick(np), c = pick(nc), t = pick(nt), f = pick(fmt), a = pick(acc);
        const int m = pick(mabs), ti = pick(tile), w = pick(win), st = pick(stg), v = pick(var);
        xc::Plan pl;
        std::string err;
        const int rc = xc::make_plan(s, p, c, t, f, a, m, ti, &pl, &err, w, st, v);
        if (rc != XCORR_OK) {
            check(!err.empty(), "error without a message", rc);
            continue;
        }
        ++nok;
        const int64_t nin = (int64_t)s * p;
        check(pl.nin == nin, "nin", pl.nin, nin);
        check(pl.nwindows == (t > 0 ? (t + pl.window - 1) / pl.window : 0), "window count", pl.nwindows, t);
        if (f != IN_CF32) {
            const int64_t lim = xc::window_limit(f, a, pl.max_abs);
            check(lim > 0 && pl.window <= lim, "window within the exact limit", pl.window, lim);
        }
        if (w > 0 && t > w) check(pl.window == w, "requested window", pl.window, w);
        check(pl.useful_cmacs == nin * (nin + 1) / 2 * c * (int64_t)t, "useful work", pl.useful_cmacs);
        check(pl.computed_cmacs >= pl.useful_cmacs, "computed >= useful", pl.computed_cmacs, pl.useful_cmacs);
        check(pl.in_bytes == (size_t)t * c * nin * xc::in_sample_bytes(f), "input bytes", (long long)pl.in_bytes);
        const size_t nbl = (size_t)s * (s + 1) / 2;
        check(pl.out_bytes == (size_t)c * nbl * p * p * xc::out_value_bytes(pl.out_dtype), "output bytes",
              (long long)pl.out_bytes);
        check(pl.variant >= 0 && pl.variant < xc::kernel_variants(pl.tile, a), "variant", pl.variant, pl.tile);
        check(pl.tile == 64 || pl.tile == 128 || pl.tile == 256 || pl.tile == 512, "tile", pl.tile);
        if (ti) check(pl.tile == ti, "tile override", pl.tile, ti);
        if (pl.tile == 256) check(xc::chan_kernel_ok(pl.nin, f, a), "whole-channel kernel accepts the job", pl.nin);
        if (pl.tile == 512) check(xc::super_kernel_ok(pl.nin, c, pl.window, f, a, pl.max_abs), "super-tiles accept", pl.nin);
        if (a == ACC_I8 && f != IN_CF32)
            check(pl.out_dtype == (pl.nwindows > 1 ? OUT_CI64 : OUT_CI32), "int8 output type", pl.out_dtype);
    }
    check(nok > 1000, "enough valid plans", nok);
    printf("plans: %d accepted\n", nok);
}

void windows()
{
    for (int f = -1; f <= 3; ++f)
        for (int a = -1; a <= 6; ++a)
            for (int m = -1; m <= 130; ++m) {
                const int64_t lim = xc::window_limit(f, a, m);
                if (lim <= 0) continue;
                if (f == IN_CF32) continue;
                const int64_t per = 2 * (int64_t)m * m;
                const int64_t cap = a == ACC_I8 ? INT32_MAX : ((int64_t)1 << 24);
                check(lim * per <= cap && (lim + 1) * per > cap, "window limit is the largest exact one", lim, m);
            }
}

void tiles()
{
    for (int64_t g = 0; g < 2000000; ++g) {
        int64_t bx = -1, by = -1;
        xc::tile_coords(g, &bx, &by);
        check(bx >= 0 && bx <= by && by * (by + 1) / 2 + bx == g, "tile coords", g, by);
    }
    for (int k = 0; k < 20000; ++k) {
        const int64_t g = (int64_t)(next_u64() >> 22);  // up to 2^42
        int64_t bx = -1, by = -1;
        xc::tile_coords(g, &bx, &by);
        check(bx >= 0 && bx <= by && by * (by + 1) / 2 + bx == g, "tile coords (large)", g, by);
    }
}

void tune_cache(const char *dir)
{
    xc::tune_clear();
    for (int k = 0; k < 200; ++k) {
        xc::TuneKey key{k % 2 ? "gfx950" : "gfx942", 1 + k, 1 + k % 2, k % 13, k % 17, k % 2, 1 + k % 5, 8, k % 3};
        static const int tl[] = {64, 128, 256, 512};
        const int tile = tl[k % 4];
        xc::TuneVal v{tile, (tile <= 128) ? k % 2 : 0, tile == 256 ? k % 4 : (tile == 512 ? k % 2 : 0), 1.5 * k};
        xc::tune_record(key, v);
    }
    std::string err;
    const std::string path = std::string(dir) + "/tune_cache.jsonl";
    const int nw = xc::tune_save(path.c_str(), &err);
    check(nw == 200, "saved entries", nw);
    xc::tune_clear();
    const int nr = xc::tune_load(path.c_str(), &err);
    check(nr == 200, "loaded entries", nr);
    for (int k = 0; k < 200; ++k) {
        xc::TuneKey key{k % 2 ? "gfx950" : "gfx942", 1 + k, 1 + k % 2, k % 13, k % 17, k % 2, 1 + k % 5, 8, k % 3};
        xc::TuneVal v{};
        check(xc::tune_lookup(key, &v) && v.us == 1.5 * k, "lookup after reload", k);
    }
    // malformed files are refused whole, without touching the cache
    static const char *bad[] = {
        "{\"arch\": \"gfx950\", \"nstation\": 1}\n",
        "garbage\n",
        "{\"arch\": \"gfx950\", \"nstation\": 4, \"npol\": 2, \"nchan_log2\": 3, \"ntime_log2\": 4, \"in\": 0, "
        "\"acc\": 1, \"max_abs\": 8, \"window\": 0, \"tile\": 96, \"staging\": 0, \"variant\": 0, \"us\": 1.0}\n",
        "{\"arch\": \"aaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaa"
        "aaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaaa\", \"nstation\": 4}\n",
    };
    for (const char *text : bad) {
        FILE *f = fopen(path.c_str(), "w");
        fputs(text, f);
        fclose(f);
        check(xc::tune_load(path.c_str(), &err) == -1 && !err.empty(), "malformed cache refused");
    }
    {
        // a line longer than the reader's buffer
        FILE *f = fopen(path.c_str(), "w");
        for (int i = 0; i < 3000; ++i) fputc('x', f);
        fputc('\n', f);
        fclose(f);
        check(xc::tune_load(path.c_str(), &err) == -1, "overlong line refused");
    }
    check(xc::tune_load((std::string(dir) + "/missing/none.jsonl").c_str(), &err) == -1, "missing file");
    xc::TuneVal v{};
    xc::TuneKey key{"gfx950", 2, 2, 1, 1, 1, 2, 8, 1};
    check(xc::tune_lookup(key, &v), "cache kept after refused loads");
    for (int64_t n = -3; n < 5000; ++n) {
        const int c = xc::size_class(n);
        check(n <= 1 ? c == 0 : (((int64_t)1 << c) >= n && ((int64_t)1 << (c - 1)) < n), "size class", n, c);
    }
}

}  // namespace

int main(int argc, char **argv)
{
    const char *dir = argc > 1 ? argv[1] : ".";
    plans();
    windows();
    tiles();
    tune_cache(dir);
    if (g_fail) {
        fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    printf("ok\n");
    return 0;
}
