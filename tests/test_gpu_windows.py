"""GPU parity of the accumulation windows (Sec. 2.3: accumulators wider than the data, dumped
before they can overflow) against the oracle, on every kernel.

* Worst-amplitude inputs at the exact window limit T_d and at T_d + 1: one window (ci32 /
  c64 output) and two windows summed into int64 / fp64 (ci64 / c128), for int32
  accumulators (8-bit samples at +-127, 4-bit samples scaled by 8 on the super-tiles) and
  fp32 accumulators (8-bit samples at -128 on the fp16 / FP32 paths, 4-bit samples at -8 on
  the fp8 path).  The autocorrelations reach the accumulator bound exactly.
* Short windows requested by the caller (xcorr_set_window): several windows per item,
  summed with atomics into the wide output, compared bit for bit with the oracle.
"""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, device, low_dist, low_max_abs, say

pytestmark = pytest.mark.gpu


def _check(got, want, label):
    g = as_exact_int(got)
    if not np.array_equal(g, want):
        bad = np.argwhere(g != want)
        say(label, "MISMATCH count", len(bad), "first", bad[:5].tolist(),
            "got", g[tuple(bad[0])], "want", want[tuple(bad[0])])
    assert np.array_equal(g, want), label


def _run(x, ns, npol, fmt, acc, tile=None, max_abs=None, window=None):
    """One job through the C ABI; returns (numpy output, out_type, plan tile)."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    c = X.Correlator(ns, npol, x.shape[1], x.shape[0], fmt, acc, max_abs=max_abs, tile=tile, window=window)
    if tile is not None:
        assert c.tile == tile
    out = c.run(xt)
    torch.cuda.synchronize()
    res, ot, t = out.cpu().numpy(), c.out_type, c.tile
    c.close()
    del xt, out
    return res, ot, t


def rotating_worst_ci8(T, F, nin):
    """|component| = 127 everywhere: input k is b_k i^t with b_k = -127 - 127i (k even) or
    -127 + 127i (k odd).  Every autocorrelation is 2 * 127^2 per sample and every cross
    product between an even and an odd input has one part of magnitude 2 * 127^2."""
    b = np.where((np.arange(nin) % 2 == 0)[:, None], np.array([-127, -127]), np.array([-127, 127]))
    out = np.empty((T, F, nin, 2), dtype=np.int8)
    v = b.astype(np.int64)
    for r in range(4):  # multiply by i: (a, b) -> (-b, a)
        out[r::4] = v.astype(np.int8)[None, None]
        v = np.stack([-v[:, 1], v[:, 0]], axis=1)
    return out


def constant_worst(T, F, nin, lo, hi):
    """Input k constant in time: lo + lo i (k even) or lo + hi i (k odd); the even inputs'
    autocorrelations are 2 lo^2 per sample, the largest the format allows."""
    b = np.where((np.arange(nin) % 2 == 0)[:, None], np.array([lo, lo]), np.array([lo, hi]))
    return np.broadcast_to(b.astype(np.int8)[None, None], (T, F, nin, 2)).copy()


# --------------------------------------------------------------- int32 accumulators, 8-bit


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_int8_window_bound_small(oracle_mod, tile):
    """8 inputs at +-127 on the int8 path: T = 66572 fits one int32 window (the
    autocorrelations reach 2,147,479,576 <= 2^31 - 1); T = 66573 needs two (int64 totals)."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F = 4, 2, 2
    lim = X.xcorr_window_limit(X.IN_CI8, X.ACC_I8_MMA_I32, 127)
    assert lim == 66572 and lim * 2 * 127**2 <= 2**31 - 1 < (lim + 1) * 2 * 127**2
    for T, want_type in ((lim, X.OUT_CI32), (lim + 1, X.OUT_CI64)):
        x = rotating_worst_ci8(T, F, ns * npol)
        say("int8 window bound", tile, T)
        got, ot, _ = _run(x, ns, npol, "ci8", "i8", tile=tile)
        assert ot == want_type
        want = oracle_mod.xcorr(x, ns, npol)
        assert int(want[..., 0].max()) == T * 2 * 127**2
        _check(got, want, f"int8-bound/{tile}/{T}")


def test_int8_window_bound_super(oracle_mod):
    """The same bound on 8-bit super-tiles (272 inputs: a full and a partial super-row)."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F = 136, 2, 1
    for T, want_type in ((66572, X.OUT_CI32), (66573, X.OUT_CI64)):
        x = rotating_worst_ci8(T, F, ns * npol)
        say("int8 window bound super", T)
        got, ot, _ = _run(x, ns, npol, "ci8", "i8", tile=512)
        assert ot == want_type
        _check(got, oracle_mod.xcorr(x, ns, npol), f"int8-bound/super/{T}")


# --------------------------------------------------------------- fp32 accumulators, 8-bit


@pytest.mark.parametrize("acc,tile", [("f16", 64), ("f16", 128), ("f16", 256), ("f32", 64), ("f32m", 64),
                                      ("f32m", 128)])
def test_fp32_window_bound_ci8(oracle_mod, acc, tile):
    """-128 - 128i with max_abs 128: T = 512 puts the autocorrelations at 2^24 exactly (one
    fp32 window, c64); T = 513 needs two windows (fp64 totals, c128)."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F = 4, 2, 2
    lim = X.xcorr_window_limit(X.IN_CI8, X.ACC_NAMES[acc], 128)
    assert lim == 512
    for T, want_type in ((lim, X.OUT_C64), (lim + 1, X.OUT_C128)):
        x = constant_worst(T, F, ns * npol, -128, 127)
        say("fp32 window bound", acc, tile, T)
        got, ot, _ = _run(x, ns, npol, "ci8", acc, tile=tile, max_abs=128)
        assert ot == want_type
        want = oracle_mod.xcorr(x, ns, npol)
        assert int(want[..., 0].max()) == T * 2 * 128**2
        _check(got, want, f"fp32-bound/{acc}/{tile}/{T}")


# --------------------------------------------------------------- 4-bit samples


def _pack(v):
    return synth.pack_ci4(v)


def constant_worst_ci4(T, F, nin):
    """constant_worst(T, F, nin, -8, 7) packed as 4-bit samples (one row packed, then
    repeated)."""
    row = synth.pack_ci4(constant_worst(1, 1, nin, -8, 7))
    return np.broadcast_to(row, (T, F, nin)).copy()


@pytest.mark.parametrize("tile", [64, 512])
def test_fp6_window_bound_ci4(oracle_mod, tile):
    """4-bit samples at -8 - 8i on the fp6 path: T = 131072 (one fp32 window, c64) and
    T = 131073 (two windows, c128); 64-tiles and super-tiles (units from the pre-pass)."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F = (4, 2, 1) if tile == 64 else (136, 2, 1)
    lim = X.xcorr_window_limit(X.IN_CI4, X.ACC_F6E3M2_MMA_F32, 8)
    assert lim == 131072
    for T, want_type in ((lim, X.OUT_C64), (lim + 1, X.OUT_C128)):
        x = constant_worst_ci4(T, F, ns * npol)
        say("fp6 window bound", tile, T)
        got, ot, t = _run(x, ns, npol, "ci4", "f6", tile=tile)
        assert ot == want_type and t == tile
        want = oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CI4)
        assert int(want[..., 0].max()) == T * 128
        _check(got, want, f"fp6-bound/{tile}/{T}")


@pytest.mark.parametrize("tile", [64, 512])
def test_fp8_window_bound_ci4(oracle_mod, tile):
    """4-bit samples at -8 - 8i on the fp8 path: T = 131072 puts the autocorrelations at
    2^24 (one window, c64), T = 131073 needs two (c128); 64-tiles and super-tiles."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F = (4, 2, 1) if tile == 64 else (136, 2, 1)
    lim = X.xcorr_window_limit(X.IN_CI4, X.ACC_F8E4M3_MMA_F32, 8)
    assert lim == 131072
    for T, want_type in ((lim, X.OUT_C64), (lim + 1, X.OUT_C128)):
        x = constant_worst_ci4(T, F, ns * npol)
        say("fp8 window bound", tile, T)
        got, ot, _ = _run(x, ns, npol, "ci4", "f8", tile=tile)
        assert ot == want_type
        want = oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CI4)
        assert int(want[..., 0].max()) == T * 128
        _check(got, want, f"fp8-bound/{tile}/{T}")


def test_int8_ci4_window_bound_tiles(oracle_mod):
    """4-bit samples at -8 - 8i on the int8 path (unscaled operands, 64-tiles): T =
    16777215 fits one int32 window, T = 16777216 needs two."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F = 4, 2, 1
    lim = X.xcorr_window_limit(X.IN_CI4, X.ACC_I8_MMA_I32, 8)
    assert lim == 16777215
    for T, want_type in ((lim, X.OUT_CI32), (lim + 1, X.OUT_CI64)):
        x = constant_worst_ci4(T, F, ns * npol)
        say("int8 ci4 window bound", T)
        got, ot, _ = _run(x, ns, npol, "ci4", "i8", tile=64)
        assert ot == want_type
        _check(got, oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CI4), f"int8-ci4-bound/{T}")


def test_int8_ci4_window_bound_super(oracle_mod):
    """4-bit samples on the int8 super-tiles carry operands 8 x the samples, 16 x on the row
    side of a rectangle: -8 - 8i gives 2 * 128 * 64 = 16384 per sample there, so windows hold
    at most 131071 samples (2^31 - 16384 at the bound).  T = 131071 in one window on
    super-tiles; T = 131072 runs two requested windows of 131071 samples (int64 totals)."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F = 136, 2, 1
    lim = (2**31 - 1) // (256 * 8 * 8)
    assert lim == 131071 and lim * 16384 <= 2**31 - 1 < (lim + 1) * 16384
    for T, window, want_type in ((lim, None, X.OUT_CI32), (lim + 1, lim, X.OUT_CI64)):
        x = constant_worst_ci4(T, F, ns * npol)
        say("int8 ci4 super window bound", T, window)
        got, ot, t = _run(x, ns, npol, "ci4", "i8", tile=512, window=window)
        assert ot == want_type and t == 512
        _check(got, oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CI4), f"int8-ci4-super-bound/{T}")


# --------------------------------------------------------------- requested short windows


CASES = [
    # (fmt, acc, nstation, npol, tile)
    ("ci8", "i8", 128, 2, 256),    # whole channel
    ("ci8", "f16", 128, 2, 256),
    ("ci8", "i8", 100, 2, 128),    # 128-tiles, ragged
    ("ci8", "f16", 100, 2, 128),
    ("ci8", "f8", 30, 2, 64),
    ("ci8", "f32", 45, 2, 64),     # FP32 CMAC
    ("ci8", "i8", 256, 2, 512),    # 8-bit super-tiles
    ("ci4", "i8", 256, 2, 512),    # 4-bit super-tiles (scaled operands)
    ("ci4", "f8", 136, 2, 512),    # partial last super-row
    ("ci4", "i8", 70, 1, 128),
    ("ci8", "f32m", 45, 2, 128),   # fp32 matrix cores
    ("ci4", "f6", 70, 2, 128),     # fp6 e3m2
    ("ci4", "f6", 136, 2, 512),    # fp6 super-tiles (windows of whole blocks only)
    ("ci8", "f6", 33, 2, 64),
]


@pytest.mark.parametrize("window", [33, 64])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c)))
def test_requested_windows_match_oracle(oracle_mod, case, window):
    """200 samples integrated in windows of 33 (ragged) or 64 samples: 7 or 4 window sums
    per item, added into the wide output; bit-exact against the oracle."""
    from paper_1107_4264_amd import xcorr as X

    fmt, acc, ns, npol, tile = case
    F, T = 3, 200
    if fmt == "ci4":
        x = _pack(synth.voltages_np(synth.SEED_BASE + 90 + ns + window, T, F, ns * npol, ("uniform", -8, 7)))
        want = oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CI4)
    else:
        dist = low_dist(acc, ("gauss", 50.0, 127))
        x = synth.voltages_np(synth.SEED_BASE + 91 + ns + window, T, F, ns * npol, dist)
        want = oracle_mod.xcorr(x, ns, npol)
    say("requested windows", case, window)
    if acc == "f6" and tile == 512 and window % 32:
        # fp6 super-tiles take windows of whole 32-sample blocks only: refused
        with pytest.raises(X.XcorrError):
            _run(x, ns, npol, fmt, acc, tile=tile, window=window)
        return
    # 8-bit samples on the fp8 path need a declared bound of at most 16
    ma = low_max_abs(acc) if fmt == "ci8" else None
    got, ot, t = _run(x, ns, npol, fmt, acc, tile=tile, window=window, max_abs=ma)
    assert t == tile
    assert ot == (X.OUT_CI64 if acc == "i8" else X.OUT_C128)
    _check(got, want, f"windows/{case}/{window}")


def test_window_longer_than_limit_is_refused():
    from paper_1107_4264_amd import xcorr as X

    device()
    c = X.Correlator(8, 2, 2, 1000, "ci8", "f16")
    with pytest.raises(X.XcorrError) as e:
        X.xcorr_set_window(c.h, 513)
    assert e.value.code == X.ERR_UNSUPPORTED
    X.xcorr_set_window(c.h, 512)
    c.close()


@pytest.mark.parametrize("acc", ["i8", "f16"])
def test_stream_requested_windows(oracle_mod, acc):
    """A streaming integration with windows shorter than its chunks: every chunk adds
    several window sums into the totals."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    device()
    ns, npol, F, chunk, nchunk = 128, 2, 3, 96, 3
    x = synth.voltages_np(synth.SEED_BASE + 95, chunk * nchunk, F, ns * npol, ("gauss", 60.0, 127))
    st = X.Stream(ns, npol, F, chunk, "ci8", acc, window=40)
    chunks = [torch.from_numpy(np.ascontiguousarray(x[c * chunk:(c + 1) * chunk])).pin_memory()
              for c in range(nchunk)]
    out = st.begin()
    for ch in chunks:
        st.push(ch)
    st.end()
    _check(out.cpu().numpy(), oracle_mod.xcorr(x, ns, npol), f"stream-windows/{acc}")
    st.close()
