// Host-side planner: tile geometry, accumulation windows, output type and work accounting.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>

namespace xc {

struct Plan {
    int nstation = 0, npol = 0, nchan = 0, ntime = 0;
    int in_fmt = 0, acc = 0, max_abs = 0;
    int nin = 0, tile = 0, ntile_side = 0, tiles_per_chan = 0;
    int window = 0, nwindows = 0, out_dtype = 0;
    int window_req = 0;  // window the caller asked for (0: the longest exact one)
    int staging = 0;     // 0: operands staged in LDS; 1: loaded per wave through the caches
    int variant = 0;     // compile-time variant of the whole-channel (0..3, fp16 0..7) / super-tiled (0..3) kernel
    int64_t nitems = 0, useful_cmacs = 0, computed_cmacs = 0;
    size_t in_bytes = 0, out_bytes = 0;
};

// Largest exact window in samples (INT64_MAX when unbounded), or -1 on a bad argument.
int64_t window_limit(int in_fmt, int acc, int max_abs);

// Default component bound of a sample format for an arithmetic path.
int default_max_abs(int in_fmt, int acc);

// Fill `pl`.  tile_override 0 picks the default tile; window_req 0 integrates in the longest
// exact windows, a positive value in windows of that many samples (at most the exact limit);
// staging 1 runs the tiled kernel without its LDS stage (tiles 64 / 128, matrix-core paths).
// Returns an XCORR_* code and sets *err on failure.
int make_plan(int nstation, int npol, int nchan, int ntime, int in_fmt, int acc, int max_abs,
              int tile_override, Plan *pl, std::string *err, int window_req = 0, int staging = 0,
              int variant = 0);

// Number of compile-time variants of the kernel a tile value selects (1 for the tiled and
// FP32 CMAC kernels).
int kernel_variants(int tile, int acc);

// Tile value of the whole-channel kernel: one workgroup holds the triangle of up to 256
// inputs of a channel.
constexpr int CHAN_TILE = 256;

// Whether the whole-channel kernel accepts a job of nin inputs.
bool chan_kernel_ok(int nin, int in_fmt, int acc);

// Tile value of the super-tiled kernel: 256-input triangles and 256 x 128 rectangles of
// arrays of 272..2048 inputs (4-bit samples on the int8 and fp8 paths, 8-bit samples on the
// int8 path).
constexpr int SUPER_TILE = 512;

// Whether the super-tiled kernel accepts a job: CI4 samples on the int8 or fp8 path or CI8
// samples on the int8 path, nin a multiple of 16 in 272..2048; for CI4 on the int8 path
// also windows within the exact limit of its scaled operands (floor((2^31-1)/(256 m^2))
// samples for samples bounded by m).
bool super_kernel_ok(int nin, int nchan, int64_t window, int in_fmt, int acc, int max_abs);

// Exact inverse of g = by*(by+1)/2 + bx, 0 <= bx <= by.
void tile_coords(int64_t g, int64_t *bx, int64_t *by);

// Complex MACs the kernels execute per channel and sample for a tile geometry.
int64_t computed_pairs_per_sample(int nin, int tile, int acc);

// Bytes per sample of an input format; bytes per complex value of an output type.
size_t in_sample_bytes(int in_fmt);
size_t out_value_bytes(int out_dtype);

}  // namespace xc
