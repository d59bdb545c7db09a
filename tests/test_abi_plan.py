"""Host-side checks of the C ABI (no GPU): the library loads and exports every function the
header declares; the planner's tile numbering, accumulation windows, output types, work
accounting and argument checks."""

from __future__ import annotations

import ctypes
import json
import os
import subprocess

import pytest

from paper_1107_4264_amd import xcorr as X

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_exports_every_header_function():
    names = X.header_functions()
    assert "xcorr_create" in names and "xcorr_run" in names
    out = subprocess.run(["nm", "-D", "--defined-only", X.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, f"not exported: {missing}"
    for n in names:
        assert hasattr(X.lib(), n)


def test_tile_coords_exhaustive():
    """Triangular numbering g = by(by+1)/2 + bx with bx <= by (Sec. 4.2), inverted exactly,
    checked against enumeration for every g < 2^21 and at large g."""
    g = 0
    for by in range(2048):
        for bx in range(by + 1):
            if g % 97 == 0 or by < 64:
                assert X.xcorr_tile_coords(g) == (bx, by)
            g += 1
    for by in [10**6, 2**31 - 1, 3 * 10**9]:
        base = by * (by + 1) // 2
        assert X.xcorr_tile_coords(base) == (0, by)
        assert X.xcorr_tile_coords(base + by) == (by, by)
        assert X.xcorr_tile_coords(base - 1) == (by - 1, by - 1)
    with pytest.raises(X.XcorrError):
        X.xcorr_tile_coords(-1)


def test_window_limits():
    # int32 accumulators, 8-bit samples within [-127, 127]: floor((2^31-1) / (2*127^2))
    assert X.xcorr_window_limit(X.IN_CI8, X.ACC_I8_MMA_I32, 127) == 66572
    # fp32 accumulators: floor(2^24 / (2 m^2))
    assert X.xcorr_window_limit(X.IN_CI8, X.ACC_F16_MMA_F32, 128) == 512
    assert X.xcorr_window_limit(X.IN_CI8, X.ACC_F32_CMAC, 127) == 520
    assert X.xcorr_window_limit(X.IN_CI4, X.ACC_F8E4M3_MMA_F32, 8) == 131072
    assert X.xcorr_window_limit(X.IN_CI4, X.ACC_I8_MMA_I32, 8) == 16777215
    assert X.xcorr_window_limit(X.IN_CI8, X.ACC_F16_MMA_F32, 18) == 25890
    with pytest.raises(X.XcorrError):
        X.xcorr_window_limit(X.IN_CI8, X.ACC_I8_MMA_I32, 128)  # -128 cannot be negated in int8
    with pytest.raises(X.XcorrError):
        X.xcorr_window_limit(X.IN_CI4, X.ACC_I8_MMA_I32, 9)


def test_window_bound_is_tight_for_ci4():
    """4-bit worst case per sample is 2*8^2 = 128 (an autocorrelation of -8 - 8i)."""
    assert (-8) * (-8) + (-8) * (-8) == 128
    assert X.xcorr_window_limit(X.IN_CI4, X.ACC_F16_MMA_F32, 8) * 128 == 2**24


@pytest.mark.parametrize("acc", [X.ACC_F32_CMAC, X.ACC_I8_MMA_I32, X.ACC_F16_MMA_F32])
def test_plan_windows_and_types(acc):
    p = X.xcorr_plan(128, 2, 1024, 1000, X.IN_CI8, acc, 18)
    assert p["nwindows"] == 1
    assert p["out_dtype"] == (X.OUT_CI32 if acc == X.ACC_I8_MMA_I32 else X.OUT_C64)
    p = X.xcorr_plan(128, 2, 4, 70000, X.IN_CI8, acc, 0)
    if acc == X.ACC_I8_MMA_I32:
        assert p["nwindows"] == 2 and p["out_dtype"] == X.OUT_CI64
        assert p["window"] % 64 == 0 and p["window"] <= 66572
    else:
        assert p["nwindows"] > 1 and p["out_dtype"] == X.OUT_C128
        assert p["window"] * 2 * p["max_abs"] ** 2 <= 2**24


def test_plan_sizes_config_shapes():
    # 32 stations x 2 pol, 16 channels, 256 samples: 2080 input pairs (Eq. 5), 528 baselines
    p = X.xcorr_plan(32, 2, 16, 256, X.IN_CI8, X.ACC_F32_CMAC, 8)
    assert p["nin"] == 64
    assert p["useful_cmacs"] == 2080 * 16 * 256
    assert p["in_bytes"] == 256 * 16 * 64 * 2
    assert p["out_bytes"] == 16 * 528 * 4 * 8
    # 128 stations x 2 pol at 1024 channels: one whole-channel item per channel by default,
    # three 128-tiles per channel on request; the same 36 blocks of 32x32 pairs either way
    # (16 + 10 + 10 for the tiles)
    p = X.xcorr_plan(128, 2, 1024, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 18)
    assert (p["tile"], p["ntile_side"], p["tiles_per_chan"], p["nitems"]) == (256, 1, 1, 1024)
    assert p["computed_cmacs"] == 36 * 1024 * 1024 * 1000
    p = X.xcorr_plan(128, 2, 1024, 1000, X.IN_CI8, X.ACC_F16_MMA_F32, 18, 128)
    assert (p["tile"], p["ntile_side"], p["tiles_per_chan"], p["nitems"]) == (128, 2, 3, 3072)
    assert p["computed_cmacs"] == 36 * 1024 * 1024 * 1000
    # 512 stations x 2 pol, 4-bit: 16 super-tile pieces per channel (36 tiles of 128)
    p = X.xcorr_plan(512, 2, 256, 4096, X.IN_CI4, X.ACC_I8_MMA_I32, 0)
    assert p["tiles_per_chan"] == 16 and p["nwindows"] == 1 and p["out_dtype"] == X.OUT_CI32
    assert X.xcorr_plan(512, 2, 256, 4096, X.IN_CI4, X.ACC_I8_MMA_I32, 0, 128)["tiles_per_chan"] == 36
    assert p["in_bytes"] == 4096 * 256 * 1024


def test_waste_factor_matches_paper():
    """With whole diagonal tiles computed (the paper's kernel), computed / useful work is
    2(N + RT) / (2N + 1) for N dual-pol stations and tiles of RT stations (Sec. 6.1)."""
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as fh:
        gold = json.load(fh)["waste_factor"]
    for N in gold["stations"]:
        p = X.xcorr_plan(N, 2, 1, 1, X.IN_CI8, X.ACC_F32_CMAC, 0)
        RT = p["tile"] // 2
        ratio = p["computed_cmacs"] / p["useful_cmacs"]
        assert ratio == pytest.approx(2 * (N + RT) / (2 * N + 1), rel=1e-12)


def test_diagonal_skip_reduces_waste():
    p = X.xcorr_plan(128, 2, 1, 1, X.IN_CI8, X.ACC_F16_MMA_F32, 0)
    assert p["useful_cmacs"] / p["computed_cmacs"] == pytest.approx(32896 / 36864)


@pytest.mark.parametrize("args,code", [
    ((0, 2, 1, 1, X.IN_CI8, X.ACC_F16_MMA_F32, 0), X.ERR_INVALID_ARG),
    ((4, 3, 1, 1, X.IN_CI8, X.ACC_F16_MMA_F32, 0), X.ERR_INVALID_ARG),
    ((4, 2, 0, 1, X.IN_CI8, X.ACC_F16_MMA_F32, 0), X.ERR_INVALID_ARG),
    ((4, 2, 1, -1, X.IN_CI8, X.ACC_F16_MMA_F32, 0), X.ERR_INVALID_ARG),
    ((4, 2, 1, 1, 7, X.ACC_F16_MMA_F32, 0), X.ERR_INVALID_ARG),
    ((4, 2, 1, 1, X.IN_CF32, X.ACC_I8_MMA_I32, 0), X.ERR_UNSUPPORTED),
    ((4, 2, 1, 1, X.IN_CI8, X.ACC_F8E4M3_MMA_F32, 127), X.ERR_UNSUPPORTED),
    ((4, 2, 1, 1, X.IN_CI8, X.ACC_I8_MMA_I32, 128), X.ERR_INVALID_ARG),
    ((40000, 2, 1, 1, X.IN_CI8, X.ACC_I8_MMA_I32, 0), X.ERR_RANGE),
])
def test_plan_rejects(args, code):
    with pytest.raises(X.XcorrError) as ei:
        X.xcorr_plan(*args)
    assert ei.value.code == code
    assert X.last_error()


def test_fp8_accepts_small_bound_and_ci4():
    assert X.xcorr_plan(4, 2, 1, 1, X.IN_CI8, X.ACC_F8E4M3_MMA_F32, 16)["out_dtype"] == X.OUT_C64
    assert X.xcorr_plan(4, 2, 1, 1, X.IN_CI4, X.ACC_F8E4M3_MMA_F32, 0)["max_abs"] == 8


def test_empty_integration_plans_no_items():
    p = X.xcorr_plan(4, 2, 3, 0, X.IN_CI8, X.ACC_I8_MMA_I32, 0)
    assert p["nitems"] == 0 and p["out_dtype"] == X.OUT_CI32 and p["in_bytes"] == 0


def test_destroy_null_is_noop():
    X.xcorr_destroy(ctypes.c_void_p(0))
    assert X.xcorr_in_bytes(ctypes.c_void_p(0)) == 0


def test_table1_model():
    """The intensity model reproduces the paper's Table 1 from its hardware numbers."""
    from paper_1107_4264_amd import perfmodel as pm

    with open(os.path.join(GOLDEN, "paper_numbers.json")) as fh:
        gold = json.load(fh)
    hw, lv = gold["gtx480"], gold["table1"]["levels"]
    assert round(hw["peak_gflops"] / hw["device_gbps"], 1) == lv[2]["ai"]
    assert round(hw["peak_gflops"] / hw["pcie_gbps"]) == lv[3]["ai"]
    assert pm.required_square_tile(lv[1]["ai"]) == lv[0]["tile"]
    assert pm.required_square_tile(lv[2]["ai"]) == lv[1]["tile"]
    assert pm.required_square_tile(lv[3]["ai"]) == lv[2]["tile"]
    assert pm.tile_registers(1, 1) == 16
    assert pm.staging_bytes(8, 8) == lv[1]["resources_bytes"]
    assert pm.staging_bytes(210, 210) == lv[2]["resources_bytes"]
    assert pm.tile_ai(1, 1, 1, word=4.0) == pytest.approx(32 / 96)
    assert pm.tile_ai(1, 1, 1) == pytest.approx(gold["intensity"]["single_baseline_ai"])
    assert pm.tile_ai(8, 8, 1e9) == pytest.approx(8.0, rel=1e-6)


@pytest.mark.parametrize("acc", [X.ACC_I8_MMA_I32, X.ACC_F16_MMA_F32])
def test_tile_choice(acc):
    """The whole-channel kernel (tile 256) is the default for 193..256 inputs that are a
    multiple of 8 (16-byte rows), CI8 input and the int8 / fp16 paths."""
    def tile(ns, npol, t=0, fmt=X.IN_CI8, a=acc):
        return X.xcorr_plan(ns, npol, 3, 100, fmt, a, 0, t)["tile"]

    assert tile(128, 2) == 256
    assert tile(100, 2) == 256        # nin 200
    assert tile(256, 1) == 256        # single polarisation
    assert tile(96, 2) == 128         # nin 192: tiles
    assert tile(127, 2) == 128        # nin 254: rows not 16-byte aligned
    assert tile(129, 2) == 128        # nin 258
    assert tile(128, 2, fmt=X.IN_CI4) == 128
    assert tile(128, 2, a=X.ACC_F32_CMAC) == 64
    # 4-bit samples from 512 inputs (a multiple of 256): super-tiles on the int8 path
    assert tile(256, 2, fmt=X.IN_CI4) == (512 if acc == X.ACC_I8_MMA_I32 else 128)
    assert tile(512, 2, fmt=X.IN_CI4) == (512 if acc == X.ACC_I8_MMA_I32 else 128)
    assert tile(512, 2, fmt=X.IN_CI4, a=X.ACC_F8E4M3_MMA_F32) == 512
    assert tile(260, 2, fmt=X.IN_CI4) == 128
    # 8-bit samples from 512 inputs: super-tiles on the int8 path only
    assert tile(256, 2) == (512 if acc == X.ACC_I8_MMA_I32 else 128)
    assert tile(384, 2) == (512 if acc == X.ACC_I8_MMA_I32 else 128)
    assert tile(250, 2) == 128
    # explicit shapes
    assert tile(32, 2, 256) == 256    # allowed below the automatic threshold
    assert tile(128, 2, 128) == 128
    assert tile(128, 2, 64) == 64
    for bad in [(129, 2, 256), (127, 2, 256), (64, 2, 32), (64, 2, 512)]:
        with pytest.raises(X.XcorrError) as ei:
            tile(*bad)
        assert ei.value.code == X.ERR_INVALID_ARG
    with pytest.raises(X.XcorrError):
        tile(128, 2, 256, fmt=X.IN_CI4)
    with pytest.raises(X.XcorrError):
        X.xcorr_plan(128, 2, 3, 100, X.IN_CI8, X.ACC_F8E4M3_MMA_F32, 16, 256)
    with pytest.raises(X.XcorrError):
        X.xcorr_plan(128, 2, 3, 100, X.IN_CI8, X.ACC_F32_CMAC, 0, 256)


def test_whole_channel_items_and_windows():
    # one item per (channel, window); windows stay multiples of the 64-sample block
    p = X.xcorr_plan(128, 2, 10, 70000, X.IN_CI8, X.ACC_I8_MMA_I32, 0)
    assert p["tile"] == 256 and p["nwindows"] == 2 and p["window"] % 64 == 0
    assert p["nitems"] == 10 * 2 and p["out_dtype"] == X.OUT_CI64
    p = X.xcorr_plan(16, 2, 10, 100, X.IN_CI8, X.ACC_F16_MMA_F32, 0, 256)
    assert p["computed_cmacs"] == 36 * 1024 * 10 * 100


def test_super_tile_plan():
    # 1024 inputs, 4-bit samples, int8 path: 4 super-rows -> 4 triangles + 12 rectangles
    p = X.xcorr_plan(512, 2, 256, 4096, X.IN_CI4, X.ACC_I8_MMA_I32, 0, 512)
    assert p["tile"] == 512 and p["ntile_side"] == 4 and p["tiles_per_chan"] == 16
    assert p["nwindows"] == 1 and p["out_dtype"] == X.OUT_CI32
    assert p["nitems"] == 256 * 16
    # computed pairs: 4 x 36 blocks + 12 x 32 blocks of 32 x 32
    assert p["computed_cmacs"] == (4 * 36 + 12 * 32) * 1024 * 256 * 4096
    assert p["useful_cmacs"] == 1024 * 1025 // 2 * 256 * 4096
    # the operands are 8 x the samples (16 x on a rectangle's row side): one window of
    # floor((2^31-1) / (256 m^2)) samples
    lim = (2 ** 31 - 1) // (256 * 8 * 8)
    X.xcorr_plan(256, 2, 2, lim, X.IN_CI4, X.ACC_I8_MMA_I32, 0, 512)
    with pytest.raises(X.XcorrError):
        X.xcorr_plan(256, 2, 2, lim + 1, X.IN_CI4, X.ACC_I8_MMA_I32, 0, 512)
    # a smaller declared bound allows longer jobs
    X.xcorr_plan(256, 2, 2, lim + 1, X.IN_CI4, X.ACC_I8_MMA_I32, 4, 512)
    # past the scaled window the automatic choice keeps 128-tiles (same output type)
    p = X.xcorr_plan(256, 2, 2, lim + 1, X.IN_CI4, X.ACC_I8_MMA_I32, 0)
    assert p["tile"] == 128 and p["out_dtype"] == X.OUT_CI32


@pytest.mark.parametrize("args", [
    (128, 2, 4, 100, "IN_CI4", "ACC_I8_MMA_I32"),   # 256 inputs: one super-row
    (204, 2, 4, 100, "IN_CI4", "ACC_I8_MMA_I32"),   # 408 inputs: not a multiple of 16
    (1280, 2, 4, 100, "IN_CI4", "ACC_I8_MMA_I32"),  # 2560 inputs: above 2048
    (256, 2, 4, 100, "IN_CI8", "ACC_F16_MMA_F32"),  # 8-bit samples on the fp16 path
    (256, 2, 4, 100, "IN_CI4", "ACC_F16_MMA_F32"),  # fp16 path
])
def test_super_tile_rejected(args):
    ns, npol, F, T, fmt, acc = args
    with pytest.raises(X.XcorrError):
        X.xcorr_plan(ns, npol, F, T, getattr(X, fmt), getattr(X, acc), 0, 512)


def test_super_tile_f8_windows():
    # fp8 super-tiles keep the usual fp32 windows (2^24 / (2 m^2) samples, m = 8 for 4-bit)
    p = X.xcorr_plan(256, 2, 1, 131072, X.IN_CI4, X.ACC_F8E4M3_MMA_F32, 0)
    assert p["tile"] == 512 and p["nwindows"] == 1 and p["out_dtype"] == X.OUT_C64
    p = X.xcorr_plan(256, 2, 1, 131072 + 300, X.IN_CI4, X.ACC_F8E4M3_MMA_F32, 0)
    assert p["tile"] == 512 and p["nwindows"] == 2 and p["out_dtype"] == X.OUT_C128
    assert p["window"] == 131072


def test_super_tile_ci8():
    # 8-bit samples on the int8 path: super-tiles on request, usual windows
    p = X.xcorr_plan(512, 2, 4, 100, X.IN_CI8, X.ACC_I8_MMA_I32, 0, 512)
    assert p["tile"] == 512 and p["tiles_per_chan"] == 16 and p["out_dtype"] == X.OUT_CI32
    p = X.xcorr_plan(256, 2, 1, 66572 + 200, X.IN_CI8, X.ACC_I8_MMA_I32, 0, 512)
    assert p["nwindows"] == 2 and p["out_dtype"] == X.OUT_CI64
    with pytest.raises(X.XcorrError):
        X.xcorr_plan(256, 2, 4, 100, X.IN_CI8, X.ACC_F16_MMA_F32, 0, 512)


def test_super_tile_ragged():
    # any multiple of 16 above 256: the last super-row is partial (padded with zero inputs)
    p = X.xcorr_plan(200, 2, 3, 100, X.IN_CI4, X.ACC_I8_MMA_I32, 0, 512)
    assert p["ntile_side"] == 2 and p["tiles_per_chan"] == 4
    assert p["computed_cmacs"] == (2 * 36 + 2 * 32) * 1024 * 3 * 100
    # automatic choice: super-tiles only when the padding costs <= 15 % more blocks than
    # 128-tiles: 496 / 752 / 1008 inputs (last 32-block of a super-row) yes, 272 / 400 no
    def auto(nin, fmt=X.IN_CI4, acc=X.ACC_I8_MMA_I32):
        return X.xcorr_plan(nin // 2, 2, 3, 100, fmt, acc, 0)["tile"]

    assert auto(496) == 512 and auto(752) == 512 and auto(1008) == 512
    assert auto(496, X.IN_CI8) == 512 and auto(496, acc=X.ACC_F8E4M3_MMA_F32) == 512
    assert auto(272) == 128 and auto(400) == 128 and auto(784) == 128


def test_requested_windows():
    """xcorr_set_window / the window argument of xcorr_plan: windows of the requested length
    (any length up to the exact limit), several windows -> wide output; longer than the
    limit -> UNSUPPORTED; negative -> INVALID_ARG; 0 -> the longest exact window."""
    p = X.xcorr_plan(128, 2, 4, 200, X.IN_CI8, X.ACC_I8_MMA_I32, 0, 0, 33)
    assert p["window"] == 33 and p["nwindows"] == 7 and p["out_dtype"] == X.OUT_CI64
    assert p["nitems"] == 4 * p["tiles_per_chan"] * 7
    p = X.xcorr_plan(128, 2, 4, 200, X.IN_CI8, X.ACC_F16_MMA_F32, 0, 0, 200)
    assert p["nwindows"] == 1 and p["out_dtype"] == X.OUT_C64
    p = X.xcorr_plan(128, 2, 4, 200, X.IN_CI8, X.ACC_F16_MMA_F32, 0, 0, 0)
    assert p["nwindows"] == 1 and p["window"] == 200
    with pytest.raises(X.XcorrError) as e:
        X.xcorr_plan(128, 2, 4, 2000, X.IN_CI8, X.ACC_F16_MMA_F32, 0, 0, 513)
    assert e.value.code == X.ERR_UNSUPPORTED
    with pytest.raises(X.XcorrError) as e:
        X.xcorr_plan(128, 2, 4, 2000, X.IN_CI8, X.ACC_F16_MMA_F32, 0, 0, -1)
    assert e.value.code == X.ERR_INVALID_ARG
    # float samples: any window (fp64 sums of fp32 windows)
    p = X.xcorr_plan(8, 2, 1, 1000, X.IN_CF32, X.ACC_F32_CMAC, 0, 0, 100)
    assert p["nwindows"] == 10 and p["out_dtype"] == X.OUT_C128


def test_super_tiles_with_requested_windows():
    """4-bit samples on the int8 super-tiles carry 8x and 16x operands: an integration
    longer than their scaled limit (131071 samples) runs on super-tiles once windows within
    that limit are requested."""
    lim = (2**31 - 1) // (256 * 64)
    with pytest.raises(X.XcorrError):
        X.xcorr_plan(256, 2, 2, lim + 1, X.IN_CI4, X.ACC_I8_MMA_I32, 0, 512)
    p = X.xcorr_plan(256, 2, 2, lim + 1, X.IN_CI4, X.ACC_I8_MMA_I32, 0, 512, lim)
    assert p["tile"] == 512 and p["nwindows"] == 2 and p["out_dtype"] == X.OUT_CI64
    p = X.xcorr_plan(256, 2, 2, 10 * lim, X.IN_CI4, X.ACC_I8_MMA_I32, 0, 0, lim)
    assert p["tile"] == 512


def test_fp32_matrix_core_path_plans():
    """The fp32 matrix-core path: fp32 windows like the fp16 path, tiled kernel only, integer
    samples only."""
    assert X.xcorr_window_limit(X.IN_CI8, X.ACC_F32_MMA_F32, 128) == 512
    assert X.xcorr_window_limit(X.IN_CI4, X.ACC_F32_MMA_F32, 8) == 131072
    p = X.xcorr_plan(128, 2, 4, 1000, X.IN_CI8, X.ACC_F32_MMA_F32, 18)
    assert p["tile"] == 128 and p["out_dtype"] == X.OUT_C64 and p["nwindows"] == 1
    assert X.xcorr_plan(16, 2, 4, 100, X.IN_CI8, X.ACC_F32_MMA_F32, 0)["tile"] == 64
    assert X.xcorr_plan(40, 2, 4, 1100, X.IN_CI8, X.ACC_F32_MMA_F32, 0)["out_dtype"] == X.OUT_C128
    for tile in (256, 512):
        with pytest.raises(X.XcorrError):
            X.xcorr_plan(128, 2, 4, 100, X.IN_CI8, X.ACC_F32_MMA_F32, 0, tile)
    with pytest.raises(X.XcorrError) as e:
        X.xcorr_plan(8, 2, 1, 10, X.IN_CF32, X.ACC_F32_MMA_F32, 0)
    assert e.value.code == X.ERR_UNSUPPORTED


def test_fp6_path_plans():
    """fp6 e3m2 holds the integers of [-8, 8]: CI4 always, CI8 only with a declared bound of
    at most 8; fp32 windows; super-tiles for 4-bit samples above 256 inputs, else the tiled
    kernel."""
    assert X.xcorr_window_limit(X.IN_CI4, X.ACC_F6E3M2_MMA_F32, 8) == 131072
    p = X.xcorr_plan(512, 2, 256, 4096, X.IN_CI4, X.ACC_F6E3M2_MMA_F32, 0)
    assert p["tile"] == 512 and p["out_dtype"] == X.OUT_C64 and p["max_abs"] == 8
    assert X.xcorr_plan(8, 2, 1, 10, X.IN_CI8, X.ACC_F6E3M2_MMA_F32, 8)["out_dtype"] == X.OUT_C64
    with pytest.raises(X.XcorrError) as e:
        X.xcorr_plan(8, 2, 1, 10, X.IN_CI8, X.ACC_F6E3M2_MMA_F32, 9)
    assert e.value.code == X.ERR_UNSUPPORTED
    with pytest.raises(X.XcorrError):
        X.xcorr_plan(512, 2, 4, 100, X.IN_CI4, X.ACC_F6E3M2_MMA_F32, 0, 256)
    # super-tiles on request (4-bit samples): windows must start on whole 32-sample blocks,
    # and 8-bit samples stay on the tiled kernel
    q = X.xcorr_plan(512, 2, 4, 100, X.IN_CI4, X.ACC_F6E3M2_MMA_F32, 0, 512)
    assert q["tile"] == 512 and q["ntile_side"] == 4 and q["tiles_per_chan"] == 16
    assert X.xcorr_plan(512, 2, 4, 100, X.IN_CI4, X.ACC_F6E3M2_MMA_F32, 0, 512, 64)["nwindows"] == 2
    for bad in ((X.IN_CI4, 48), (X.IN_CI4, 50)):
        with pytest.raises(X.XcorrError):
            X.xcorr_plan(512, 2, 4, 100, bad[0], X.ACC_F6E3M2_MMA_F32, 0, 512, bad[1])
    with pytest.raises(X.XcorrError):
        X.xcorr_plan(512, 2, 4, 100, X.IN_CI8, X.ACC_F6E3M2_MMA_F32, 8, 512)
