// Cache of tuned kernel shapes: an in-process map from (architecture, job shape class) to
// the fastest kernel shape, with a plain JSON-lines file format for keeping it across
// processes.
#include "tune.h"

#include <stdio.h>

#include <map>
#include <mutex>
#include <tuple>

namespace xc {
namespace {

auto key_tuple(const TuneKey &k)
{
    return std::tie(k.arch, k.nstation, k.npol, k.nchan_class, k.ntime_class, k.in_fmt, k.acc, k.max_abs,
                    k.window_req);
}

struct KeyLess {
    bool operator()(const TuneKey &a, const TuneKey &b) const { return key_tuple(a) < key_tuple(b); }
};

std::mutex g_mu;
std::map<TuneKey, TuneVal, KeyLess> g_map;

bool valid_val(const TuneVal &v)
{
    const bool tile_ok = v.tile == 64 || v.tile == 128 || v.tile == 256 || v.tile == 512;
    const bool staging_ok = v.staging == 0 || (v.staging == 1 && (v.tile == 64 || v.tile == 128));
    const int nvar = v.tile == 256 ? 8 : (v.tile == 512 ? 4 : 1);
    return tile_ok && staging_ok && v.variant >= 0 && v.variant < nvar && v.us >= 0.0;
}

}  // namespace

int size_class(int64_t n)
{
    int c = 0;
    while (c < 62 && ((int64_t)1 << c) < n) ++c;
    return c;
}

bool tune_lookup(const TuneKey &k, TuneVal *v)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_map.find(k);
    if (it == g_map.end()) return false;
    *v = it->second;
    return true;
}

void tune_record(const TuneKey &k, const TuneVal &v)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_map[k] = v;
}

void tune_clear()
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_map.clear();
}

int tune_save(const char *path, std::string *err)
{
    std::lock_guard<std::mutex> lk(g_mu);
    FILE *f = fopen(path, "w");
    if (!f) {
        *err = std::string("cannot write ") + path;
        return -1;
    }
    int n = 0;
    for (const auto &kv : g_map) {
        const TuneKey &k = kv.first;
        const TuneVal &v = kv.second;
        fprintf(f,
                "{\"arch\": \"%s\", \"nstation\": %d, \"npol\": %d, \"nchan_log2\": %d, \"ntime_log2\": %d, "
                "\"in\": %d, \"acc\": %d, \"max_abs\": %d, \"window\": %d, \"tile\": %d, \"staging\": %d, "
                "\"variant\": %d, \"us\": %.3f}\n",
                k.arch.c_str(), k.nstation, k.npol, k.nchan_class, k.ntime_class, k.in_fmt, k.acc, k.max_abs,
                k.window_req, v.tile, v.staging, v.variant, v.us);
        ++n;
    }
    if (fclose(f) != 0) {
        *err = std::string("write error on ") + path;
        return -1;
    }
    return n;
}

int tune_load(const char *path, std::string *err)
{
    FILE *f = fopen(path, "r");
    if (!f) {
        *err = std::string("cannot read ") + path;
        return -1;
    }
    char line[768];
    int n = 0, lineno = 0;
    std::map<TuneKey, TuneVal, KeyLess> got;
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        bool blank = true;
        for (const char *c = line; *c; ++c)
            if (*c != ' ' && *c != '\t' && *c != '\n' && *c != '\r') blank = false;
        if (blank) continue;
        TuneKey k;
        TuneVal v;
        char arch[64] = {0};
        int used = 0;
        const int m = sscanf(line,
                             " {\"arch\": \"%63[^\"]\", \"nstation\": %d, \"npol\": %d, \"nchan_log2\": %d, "
                             "\"ntime_log2\": %d, \"in\": %d, \"acc\": %d, \"max_abs\": %d, \"window\": %d, "
                             "\"tile\": %d, \"staging\": %d, \"variant\": %d, \"us\": %lf}%n",
                             arch, &k.nstation, &k.npol, &k.nchan_class, &k.ntime_class, &k.in_fmt, &k.acc,
                             &k.max_abs, &k.window_req, &v.tile, &v.staging, &v.variant, &v.us, &used);
        if (m != 13 || used == 0 || !valid_val(v)) {
            fclose(f);
            *err = std::string(path) + ": bad entry on line " + std::to_string(lineno);
            return -1;
        }
        k.arch = arch;
        got[k] = v;
        ++n;
    }
    fclose(f);
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &kv : got) g_map[kv.first] = kv.second;
    return n;
}

}  // namespace xc
