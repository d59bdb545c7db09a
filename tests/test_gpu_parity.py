"""GPU parity: the HIP X-engine (through the C ABI) against the CPU oracle on the same seeded
inputs.  Integer-sample paths must match bit for bit; float samples on the FP32 path must
stay within the rounding bound of an fp32 sum."""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests import refmath
from tests.gpu_util import as_exact_int, device, low_dist, low_max_abs, run_xeng, say

pytestmark = pytest.mark.gpu

PATHS = ["f32", "i8", "f16", "f8", "f32m", "f6"]


def _oracle_ci8(oracle_mod, x, ns, npol, chans=None):
    return oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CI8, chans=chans)


def _check_exact(got, want, label):
    g = as_exact_int(got)
    if not np.array_equal(g, want):
        bad = np.argwhere(g != want)
        say(label, "MISMATCH count", len(bad), "first", bad[:5].tolist(),
            "got", g[tuple(bad[0])], "want", want[tuple(bad[0])])
    assert np.array_equal(g, want), label


# --------------------------------------------------------------- the small workload


@pytest.mark.parametrize("acc", PATHS)
def test_small_config_all_paths(oracle_mod, acc):
    """32 stations x 2 pol, 16 channels, 256 samples, uniform [-8, 7] (the small workload)."""
    ns, npol, F, T = 32, 2, 16, 256
    x = synth.voltages_np(synth.SEED_BASE + 0, T, F, ns * npol, ("uniform", -8, 7))
    say("small config", acc)
    got, ot = run_xeng(x, ns, npol, "ci8", acc, max_abs=8)
    _check_exact(got, _oracle_ci8(oracle_mod, x, ns, npol), f"small/{acc}")


RAGGED = [
    # (nstation, npol, nchan, ntime)
    (1, 1, 1, 1),
    (1, 2, 3, 5),
    (3, 2, 2, 7),
    (17, 1, 3, 33),
    (25, 2, 5, 100),   # nin = 50: not a multiple of the load width
    (33, 2, 9, 65),    # nin = 66: tiles of 128 with padding
    (67, 1, 2, 129),   # nin = 67: odd, element loads
    (100, 2, 3, 257),  # nin = 200: two 128-tiles, ragged last tile
    (64, 2, 8, 64),    # exact tiles
]


@pytest.mark.parametrize("acc", PATHS)
@pytest.mark.parametrize("shape", RAGGED, ids=lambda s: "x".join(map(str, s)))
def test_ragged_shapes_ci8(oracle_mod, acc, shape):
    ns, npol, F, T = shape
    dist = low_dist(acc, ("gauss", 40.0, 127))
    x = synth.voltages_np(1000 + ns * 31 + T, T, F, ns * npol, dist)
    say("ragged ci8", acc, shape)
    got, _ = run_xeng(x, ns, npol, "ci8", acc, max_abs=low_max_abs(acc))
    _check_exact(got, _oracle_ci8(oracle_mod, x, ns, npol), f"ragged/{acc}/{shape}")


@pytest.mark.parametrize("acc", PATHS)
@pytest.mark.parametrize("shape", [(3, 2, 2, 9), (33, 2, 9, 65), (67, 1, 2, 40), (100, 2, 3, 130)],
                         ids=lambda s: "x".join(map(str, s)))
def test_ragged_shapes_ci4(oracle_mod, acc, shape):
    ns, npol, F, T = shape
    v = synth.voltages_np(2000 + ns + T, T, F, ns * npol, ("uniform", -8, 7))
    packed = synth.pack_ci4(v)
    say("ragged ci4", acc, shape)
    got, _ = run_xeng(packed, ns, npol, "ci4", acc)
    want = oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4)
    _check_exact(got, want, f"ci4/{acc}/{shape}")


@pytest.mark.parametrize("acc", ["f32", "f16", "i8", "f32m"])
def test_extreme_values(oracle_mod, acc):
    """Every sample at the bound of the format: -128 (or -127 on the int8 path) and 127."""
    ns, npol, F, T = 20, 2, 3, 200
    lo = -127 if acc == "i8" else -128
    w = synth.words_np(7, 0, np.arange(T * F * ns * npol * 2, dtype=np.uint64))
    x = np.where(w & 1, 127, lo).astype(np.int8).reshape(T, F, ns * npol, 2)
    say("extreme values", acc)
    got, _ = run_xeng(x, ns, npol, "ci8", acc)
    _check_exact(got, _oracle_ci8(oracle_mod, x, ns, npol), f"extreme/{acc}")


@pytest.mark.parametrize("acc,T", [("f16", 1100), ("f32", 1300), ("i8", 70000), ("f32m", 1100)])
def test_multiple_windows(oracle_mod, acc, T):
    """Integrations longer than one exact window: windows summed into int64 / fp64."""
    ns, npol, F = 5, 2, 2
    x = synth.voltages_np(3000 + T, T, F, ns * npol, ("gauss", 90.0, 127))
    say("windows", acc, T)
    got, ot = run_xeng(x, ns, npol, "ci8", acc)
    from paper_1107_4264_amd import xcorr as X

    assert ot in (X.OUT_CI64, X.OUT_C128)
    _check_exact(got, _oracle_ci8(oracle_mod, x, ns, npol), f"windows/{acc}")


@pytest.mark.parametrize("acc", PATHS)
def test_empty_integration_gives_zeros(acc):
    import torch

    from paper_1107_4264_amd import xcorr as X

    say("empty", acc)
    dev = device()
    c = X.Correlator(6, 2, 3, 0, "ci4", acc)
    out = c.empty_out(dev).fill_(7)
    xin = torch.empty(0, dtype=torch.uint8, device=dev)
    X.xcorr_run(c.h, None, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert int((out != 0).sum()) == 0
    del xin
    c.close()


@pytest.mark.parametrize("T", [300, 1000])
def test_cf32_within_fp32_bound(oracle_mod, T):
    """Float samples on the FP32 path: max |error| on the Cauchy-Schwarz scale,
    |V_ij - oracle| / sqrt(|V_ii| |V_jj|) (autocorrelations of the two inputs' polarisations),
    is at most 1e-6; also every value within the rounding bound of the two-level fp32 sum
    (gamma_{2 TB + T/TB} times the magnitude sum, TB = 16 samples per block)."""
    ns, npol, F = 40, 2, 4
    rng = np.random.default_rng(11 + T)
    x = rng.standard_normal((T, F, ns * npol, 2)).astype(np.float32)
    say("cf32", T)
    got, _ = run_xeng(x, ns, npol, "cf32", "f32")
    want = oracle_mod.xcorr(x, ns, npol, fmt=oracle_mod.CF32)
    err = np.abs(refmath.as_complex_out(got) - refmath.as_complex_out(want))  # [F][nbl][npp]
    # autocorrelation of every input: slot (p, p) of baseline (s, s)
    s1, s2 = np.tril_indices(ns)
    auto_bl = np.flatnonzero(s1 == s2)
    autos = want[:, auto_bl][..., 0]  # [F][ns][npp] real parts
    scale = np.zeros_like(err)
    for p in range(npol):
        for q in range(npol):
            a_i = autos[:, s1, p * npol + p]
            a_j = autos[:, s2, q * npol + q]
            scale[:, :, p * npol + q] = np.sqrt(a_i * a_j)
    cs = float((err / scale).max())
    big = np.abs(refmath.as_complex_out(want)) >= 1.0
    rel = float((err[big] / np.abs(refmath.as_complex_out(want))[big]).max())
    say(f"cf32 T={T}: max error / sqrt(V_ii V_jj) = {cs:.3e}; max relative error where |V| >= 1 = {rel:.3e}")
    assert cs <= 1e-6
    # magnitude sums of both parts: (|ar|+|ai|)(|br|+|bi|) per sample
    y = np.zeros_like(x)
    y[..., 0] = np.abs(x[..., 0]) + np.abs(x[..., 1])
    mag = oracle_mod.xcorr(y, ns, npol, fmt=oracle_mod.CF32)[..., 0:1]
    u = 2.0**-24
    n = 2 * 16 + (T + 15) // 16
    gamma = n * u / (1 - n * u)
    assert np.all(np.abs(got.astype(np.float64) - want) <= gamma * mag)


@pytest.mark.parametrize("acc", PATHS)
def test_deterministic(acc):
    ns, npol, F, T = 70, 2, 4, 200
    x = synth.voltages_np(99, T, F, ns * npol, ("uniform", -8, 7))
    a, _ = run_xeng(x, ns, npol, "ci8", acc, max_abs=8)
    b, _ = run_xeng(x, ns, npol, "ci8", acc, max_abs=8)
    assert np.array_equal(a, b)


def test_point_source_small(oracle_mod):
    ns, npol, F, T = 40, 2, 6, 300
    x, a, s = synth.point_source_np(0xC0FFEE, T, F, ns * npol)
    for acc in ["f32", "f16", "i8", "f32m"]:
        got, _ = run_xeng(x, ns, npol, "ci8", acc, max_abs=126)
        g = refmath.as_complex_out(as_exact_int(got))
        ac = a[:, 0] + 1j * a[:, 1]
        P = (s[..., 0].astype(np.int64) ** 2 + s[..., 1].astype(np.int64) ** 2).sum(axis=0)
        s1, s2 = np.tril_indices(ns)
        for p in range(npol):
            for q in range(npol):
                gij = ac[s1 * npol + p] * np.conj(ac[s2 * npol + q])
                assert np.array_equal(g[:, :, p * npol + q], P[:, None] * gij[None, :]), acc
