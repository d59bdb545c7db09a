// Cache of tuned kernel shapes (host-only): job shape -> tile with its measured time.
#pragma once

#include <stdint.h>

#include <string>

namespace xc {

struct TuneKey {
    int nstation, npol, nchan, ntime, in_fmt, acc, max_abs;
};

// Tile recorded for the key (0 when none).
int tune_lookup(const TuneKey &k);
void tune_record(const TuneKey &k, int tile, double us);
void tune_clear();
// One JSON object per line; returns the number of entries written / read, or -1 (I/O or
// parse error, *err set).
int tune_save(const char *path, std::string *err);
int tune_load(const char *path, std::string *err);

}  // namespace xc
