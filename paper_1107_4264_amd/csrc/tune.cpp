// Cache of tuned kernel shapes: an in-process map from job shape to the fastest tile, with
// a plain JSON-lines file format for keeping it across processes.
#include "tune.h"

#include <stdio.h>

#include <map>
#include <mutex>
#include <tuple>

namespace xc {
namespace {

struct Entry {
    int tile;
    double us;
};

auto key_tuple(const TuneKey &k)
{
    return std::make_tuple(k.nstation, k.npol, k.nchan, k.ntime, k.in_fmt, k.acc, k.max_abs);
}

struct KeyLess {
    bool operator()(const TuneKey &a, const TuneKey &b) const { return key_tuple(a) < key_tuple(b); }
};

std::mutex g_mu;
std::map<TuneKey, Entry, KeyLess> g_map;

}  // namespace

int tune_lookup(const TuneKey &k)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_map.find(k);
    return it == g_map.end() ? 0 : it->second.tile;
}

void tune_record(const TuneKey &k, int tile, double us)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_map[k] = Entry{tile, us};
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
        fprintf(f,
                "{\"nstation\": %d, \"npol\": %d, \"nchan\": %d, \"ntime\": %d, \"in\": %d, \"acc\": %d, "
                "\"max_abs\": %d, \"tile\": %d, \"us\": %.3f}\n",
                k.nstation, k.npol, k.nchan, k.ntime, k.in_fmt, k.acc, k.max_abs, kv.second.tile, kv.second.us);
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
    char line[512];
    int n = 0, lineno = 0;
    std::map<TuneKey, Entry, KeyLess> got;
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        bool blank = true;
        for (const char *c = line; *c; ++c)
            if (*c != ' ' && *c != '\t' && *c != '\n' && *c != '\r') blank = false;
        if (blank) continue;
        TuneKey k;
        Entry e;
        const int m = sscanf(line,
                             " {\"nstation\": %d, \"npol\": %d, \"nchan\": %d, \"ntime\": %d, \"in\": %d, \"acc\": %d, "
                             "\"max_abs\": %d, \"tile\": %d, \"us\": %lf}",
                             &k.nstation, &k.npol, &k.nchan, &k.ntime, &k.in_fmt, &k.acc, &k.max_abs, &e.tile, &e.us);
        if (m != 9 || (e.tile != 64 && e.tile != 128 && e.tile != 256)) {
            fclose(f);
            *err = std::string(path) + ": bad entry on line " + std::to_string(lineno);
            return -1;
        }
        got[k] = e;
        ++n;
    }
    fclose(f);
    std::lock_guard<std::mutex> lk(g_mu);
    for (const auto &kv : got) g_map[kv.first] = kv.second;
    return n;
}

}  // namespace xc
