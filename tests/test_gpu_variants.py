"""GPU parity of the kernel shapes the autotuner chooses between, against the oracle, bit
for bit: the tiled kernel without its LDS stage (operands loaded per wave through the L1 /
L2 caches, the hardware-managed cache of Sec. 4.3) on every matrix-core path, the
compile-time variants of the whole-channel kernel (ring depth, wave order) and of the
super-tiles (ring depth, rotated column operands staged in LDS), and the fp32
matrix-core path."""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, device, low_dist, low_max_abs, say

pytestmark = pytest.mark.gpu


def _run(x, ns, npol, fmt, acc, **kw):
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    c = X.Correlator(ns, npol, x.shape[1], x.shape[0], fmt, acc, **kw)
    shape = (c.tile, c.staging, c.variant)
    out = c.run(torch.from_numpy(np.ascontiguousarray(x)).to(dev))
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    c.close()
    return res, shape


def _check(got, want, label):
    g = as_exact_int(got)
    if not np.array_equal(g, want):
        bad = np.argwhere(g != want)
        say(label, "MISMATCH count", len(bad), "first", bad[:5].tolist())
    assert np.array_equal(g, want), label


CACHE_SHAPES = [
    # (nstation, npol, nchan, ntime)
    (3, 2, 2, 7),
    (17, 1, 3, 33),      # odd nin
    (33, 2, 9, 65),      # 66 inputs: ragged 128-tile
    (100, 2, 3, 257),    # 200 inputs: two tiles, ragged last time step
    (64, 2, 8, 64),
]


@pytest.mark.parametrize("acc", ["i8", "f16", "f8", "f32m", "f6"])
@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("shape", CACHE_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_cache_staging_ci8(oracle_mod, acc, tile, shape):
    ns, npol, F, T = shape
    x = synth.voltages_np(5000 + ns * 7 + T, T, F, ns * npol, low_dist(acc, ("gauss", 40.0, 127)))
    say("cache staging", acc, tile, shape)
    got, sh = _run(x, ns, npol, "ci8", acc, staging=1, tile=tile, max_abs=low_max_abs(acc))
    assert sh == (tile, 1, 0)
    _check(got, oracle_mod.xcorr(x, ns, npol), f"cache/{acc}/{tile}/{shape}")


@pytest.mark.parametrize("acc", ["i8", "f16", "f8", "f32m", "f6"])
def test_cache_staging_ci4_and_windows(oracle_mod, acc):
    """4-bit samples through the caches, and an 8-bit job in several requested windows."""
    ns, npol, F, T = 45, 2, 3, 150
    packed = synth.pack_ci4(synth.voltages_np(5100, T, F, ns * npol, ("uniform", -8, 7)))
    got, sh = _run(packed, ns, npol, "ci4", acc, staging=1)
    assert sh[1] == 1
    _check(got, oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4), f"cache-ci4/{acc}")
    x = synth.voltages_np(5101, T, F, ns * npol, low_dist(acc, ("gauss", 40.0, 127)))
    got, sh = _run(x, ns, npol, "ci8", acc, staging=1, window=40, max_abs=low_max_abs(acc))
    _check(got, oracle_mod.xcorr(x, ns, npol), f"cache-windows/{acc}")


def test_cache_staging_switches_whole_channel_jobs_to_tiles():
    from paper_1107_4264_amd import xcorr as X

    device()
    c = X.Correlator(128, 2, 4, 100, "ci8", "i8")
    assert c.tile == 256
    X.xcorr_set_staging(c.h, 1)
    assert (c.tile, c.staging) == (128, 1)
    with pytest.raises(X.XcorrError):
        X.xcorr_set_tile(c.h, 256)
    X.xcorr_set_staging(c.h, 0)
    assert c.staging == 0
    c.close()
    f = X.Correlator(8, 2, 2, 10, "ci8", "f32")
    with pytest.raises(X.XcorrError) as e:
        X.xcorr_set_staging(f.h, 1)
    assert e.value.code == X.ERR_UNSUPPORTED
    f.close()


@pytest.mark.parametrize("acc", ["i8", "f16"])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", [(128, 2, 5, 1000), (100, 2, 3, 257), (256, 1, 2, 130)],
                         ids=lambda s: "x".join(map(str, s)))
def test_chan_variants(oracle_mod, acc, variant, shape):
    ns, npol, F, T = shape
    x = synth.voltages_np(5200 + variant, T, F, ns * npol, ("gauss", 40.0, 127))
    say("chan variant", acc, variant, shape)
    got, sh = _run(x, ns, npol, "ci8", acc, tile=256, variant=variant)
    assert sh == (256, 0, variant)
    _check(got, oracle_mod.xcorr(x, ns, npol), f"chan-variant/{acc}/{variant}/{shape}")


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("fmt_acc", [("ci4", "i8"), ("ci4", "f8"), ("ci8", "i8")], ids=lambda t: "-".join(t))
@pytest.mark.parametrize("shape", [(256, 2, 2, 100), (200, 2, 2, 37), (136, 2, 3, 70)],
                         ids=lambda s: "x".join(map(str, s)))
def test_super_variant(oracle_mod, fmt_acc, shape, variant):
    """Ring depth (bit 0) and rotated column operands staged in LDS (bit 1): 512 inputs (two
    full super-rows), 400 and 272 (a partial last super-row, its rotated chunks past the
    last input zero)."""
    fmt, acc = fmt_acc
    ns, npol, F, T = shape
    v = synth.voltages_np(5300 + ns, T, F, ns * npol, ("uniform", -8, 7) if fmt == "ci4" else ("gauss", 40.0, 127))
    x = synth.pack_ci4(v) if fmt == "ci4" else v
    say("super variant", fmt, acc, shape, variant)
    got, sh = _run(x, ns, npol, fmt, acc, tile=512, variant=variant)
    assert sh == (512, 0, variant)
    want = oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CI4 if fmt == "ci4" else oracle_mod.CI8)
    _check(got, want, f"super-variant/{fmt}/{acc}/{shape}")


@pytest.mark.parametrize("shape", [(256, 2, 2, 100), (200, 2, 2, 37), (136, 2, 3, 70), (512, 1, 2, 33)],
                         ids=lambda s: "x".join(map(str, s)))
def test_super_f6_variant(oracle_mod, shape):
    """fp6 super-tiles, variant 1: the rotated row fragments made by exchanging the lane
    halves of the plain ones in registers (variant 0 reads them from LDS, the other half
    with its sign bits flipped); only 0..1 exist."""
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F, T = shape
    x = synth.pack_ci4(synth.voltages_np(5400 + ns, T, F, ns * npol, ("uniform", -8, 7)))
    say("super f6 variant", shape)
    got, sh = _run(x, ns, npol, "ci4", "f6", tile=512, variant=1)
    assert sh == (512, 0, 1)
    _check(got, oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CI4), f"super-f6-variant/{shape}")
    c = X.Correlator(ns, npol, F, T, "ci4", "f6", tile=512)
    with pytest.raises(X.XcorrError):
        X.xcorr_set_variant(c.h, 2)
    c.close()


@pytest.mark.parametrize("variant", [4, 5, 6, 7])
@pytest.mark.parametrize("shape", [(128, 2, 5, 1000), (100, 2, 3, 257), (256, 1, 2, 130)],
                         ids=lambda s: "x".join(map(str, s)))
def test_chan_f16_conversion_on_all_waves(oracle_mod, variant, shape):
    """fp16 whole-channel variants 4..7: the conversion of each block spread over all eight
    waves (with the ring-depth and wave-order bits)."""
    ns, npol, F, T = shape
    x = synth.voltages_np(5250 + variant, T, F, ns * npol, ("gauss", 40.0, 127))
    say("chan f16 variant", variant, shape)
    got, sh = _run(x, ns, npol, "ci8", "f16", tile=256, variant=variant)
    assert sh == (256, 0, variant)
    _check(got, oracle_mod.xcorr(x, ns, npol), f"chan-f16-variant/{variant}/{shape}")


def test_variant_range_checked():
    from paper_1107_4264_amd import xcorr as X

    device()
    c = X.Correlator(128, 2, 2, 10, "ci8", "f16")
    with pytest.raises(X.XcorrError):
        X.xcorr_set_variant(c.h, 8)
    i = X.Correlator(128, 2, 2, 10, "ci8", "i8")
    assert i.tile == 256
    with pytest.raises(X.XcorrError):
        X.xcorr_set_variant(i.h, 4)
    i.close()
    X.xcorr_set_tile(c.h, 128)
    with pytest.raises(X.XcorrError):
        X.xcorr_set_variant(c.h, 1)
    c.close()
