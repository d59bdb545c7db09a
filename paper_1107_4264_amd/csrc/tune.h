// Cache of tuned kernel shapes (host-only): (device architecture, job shape class) -> the
// fastest kernel shape (tile, staging, variant) with its measured time.
#pragma once

#include <stdint.h>

#include <string>

namespace xc {

// Jobs of one class share a tuned shape: the same array (stations, polarisations), sample
// format, arithmetic path, component bound and requested window, on one architecture, with
// channel and sample counts in the same power-of-two bucket.
struct TuneKey {
    std::string arch;  // e.g. "gfx950"
    int nstation, npol, nchan_class, ntime_class, in_fmt, acc, max_abs, window_req;
};

struct TuneVal {
    int tile, staging, variant;
    double us;
};

// ceil(log2(n)) for n >= 1, 0 for n <= 1.
int size_class(int64_t n);

bool tune_lookup(const TuneKey &k, TuneVal *v);
void tune_record(const TuneKey &k, const TuneVal &v);
void tune_clear();
// One JSON object per line; returns the number of entries written / read, or -1 (I/O or
// parse error, *err set).
int tune_save(const char *path, std::string *err);
int tune_load(const char *path, std::string *err);

}  // namespace xc
