"""GPU parity of the whole-channel kernel (tile 256: one persistent workgroup per compute
unit holds the triangle of a channel; samples reach LDS by direct copies and the operands
by transposing LDS reads) against the oracle, bit for bit on integer samples."""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests import refmath
from tests.gpu_util import as_exact_int, device, run_xeng, say

pytestmark = pytest.mark.gpu

ACCS = ["i8", "f16"]

SHAPES = [
    # (nstation, npol, nchan, ntime)
    (128, 2, 4, 1000),   # 256 inputs, last time block partial (1000 = 15 * 64 + 40)
    (128, 2, 3, 64),     # exactly one block
    (128, 2, 2, 1),      # a single sample
    (100, 2, 3, 257),    # 200 inputs: block row 6 partial, row 7 padding
    (256, 1, 2, 130),    # single polarisation: the generic store path
    (96, 1, 3, 77),      # 96 inputs, npol 1
    (32, 2, 5, 64),      # 64 inputs: most blocks are padding
    (4, 2, 3, 7),        # 8 inputs, the smallest row of whole 16-byte chunks
]


def _check(got, want, label):
    g = as_exact_int(got)
    if not np.array_equal(g, want):
        bad = np.argwhere(g != want)
        say(label, "MISMATCH count", len(bad), "first", bad[:5].tolist(),
            "got", g[tuple(bad[0])], "want", want[tuple(bad[0])])
    assert np.array_equal(g, want), label


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_chan_matches_oracle(oracle_mod, acc, shape):
    ns, npol, F, T = shape
    x = synth.voltages_np(synth.SEED_BASE + 40, T, F, ns * npol, ("gauss", 40.0, 127))
    say("chan", acc, shape)
    got, _ = run_xeng(x, ns, npol, "ci8", acc, tile=256)
    _check(got, oracle_mod.xcorr(x, ns, npol), f"chan/{acc}/{shape}")


@pytest.mark.parametrize("acc", ACCS)
def test_chan_extreme_values(oracle_mod, acc):
    """Full-scale samples: every product at its largest magnitude (int8 path: [-127, 127];
    fp16 path: [-128, 127])."""
    ns, npol, F, T = 128, 2, 2, 200
    lo = -127 if acc == "i8" else -128
    x = synth.voltages_np(synth.SEED_BASE + 41, T, F, ns * npol, ("uniform", lo, 127))
    x[:, :, :4] = lo  # a few inputs pinned at the extreme
    say("chan extreme", acc)
    got, _ = run_xeng(x, ns, npol, "ci8", acc, tile=256)
    _check(got, oracle_mod.xcorr(x, ns, npol), f"chan-extreme/{acc}")


# channels sampled from a walk over 700 channels: first, second and third items of
# workgroups, and the last channel
WALK_CHANS = [0, 1, 8, 9, 16, 17, 24, 31, 254, 255, 256, 257, 264, 280, 511, 512, 699]


@pytest.mark.parametrize("acc", ACCS)
@pytest.mark.parametrize("npol", [2, 1])
def test_chan_many_channels_per_workgroup(oracle_mod, acc, npol):
    """More channels than compute units: each workgroup walks several channels and copies
    the next channel's first blocks while finishing the current one."""
    ns, F, T = 256 // npol, 700, 150
    x = synth.voltages_np(synth.SEED_BASE + 42, T, F, ns * npol, ("gauss", 20.0, 127))
    say("chan walk", acc, "npol", npol, "F", F)
    got, _ = run_xeng(x, ns, npol, "ci8", acc, tile=256)
    want = oracle_mod.xcorr(x, ns, npol, chans=WALK_CHANS)
    _check(got[WALK_CHANS], want, f"chan-walk/{acc}/{npol}")


def test_chan_windows_f16(oracle_mod):
    """fp32 windows of 512 samples at the default bound, summed in fp64 on the GPU."""
    ns, npol, F, T = 128, 2, 3, 1300
    x = synth.voltages_np(synth.SEED_BASE + 43, T, F, ns * npol, ("gauss", 60.0, 127))
    say("chan windows f16")
    got, ot = run_xeng(x, ns, npol, "ci8", "f16", tile=256)
    from paper_1107_4264_amd import xcorr as X

    assert ot == X.OUT_C128
    _check(got, oracle_mod.xcorr(x, ns, npol), "chan-windows/f16")


def test_chan_windows_i8(oracle_mod):
    """int32 windows (66496 samples at the default bound) summed in int64 on the GPU."""
    ns, npol, F, T = 32, 2, 2, 70000
    x = synth.voltages_np(synth.SEED_BASE + 44, T, F, ns * npol, ("uniform", -127, 127))
    say("chan windows i8")
    got, ot = run_xeng(x, ns, npol, "ci8", "i8", tile=256)
    from paper_1107_4264_amd import xcorr as X

    assert ot == X.OUT_CI64
    _check(got, oracle_mod.xcorr(x, ns, npol), "chan-windows/i8")


@pytest.mark.parametrize("acc", ACCS)
def test_chan_equals_tiles(acc):
    """The whole-channel and the 128-tile kernels give the same bits."""
    ns, npol, F, T = 128, 2, 6, 333
    x = synth.voltages_np(synth.SEED_BASE + 45, T, F, ns * npol, ("gauss", 30.0, 127))
    a, _ = run_xeng(x, ns, npol, "ci8", acc, tile=256)
    b, _ = run_xeng(x, ns, npol, "ci8", acc, tile=128)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("acc", ACCS)
def test_chan_point_source(acc):
    """Closed form for one injected point source: V_ij = a_i conj(a_j) sum_t |s|^2."""
    ns, npol, F, T = 128, 2, 2, 500
    x, a, s = synth.point_source_np(synth.SEED_BASE + 46, T, F, ns * npol)
    got, _ = run_xeng(x, ns, npol, "ci8", acc, tile=256)
    g = refmath.as_complex_out(as_exact_int(got))
    ac = a[:, 0] + 1j * a[:, 1]
    P = (s[..., 0].astype(np.int64) ** 2 + s[..., 1].astype(np.int64) ** 2).sum(axis=0)
    s1, s2 = np.tril_indices(ns)
    for p in range(npol):
        for q in range(npol):
            gij = ac[s1 * npol + p] * np.conj(ac[s2 * npol + q])
            assert np.array_equal(g[:, :, p * npol + q], P[:, None] * gij[None, :]), (acc, p, q)


@pytest.mark.parametrize("acc", ACCS)
def test_chan_stream(oracle_mod, acc):
    """Streaming chunks through the whole-channel kernel (added into the wide totals)."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    device()
    ns, npol, F, chunk, nchunk = 128, 2, 3, 100, 4
    x = synth.voltages_np(4343, chunk * nchunk, F, ns * npol, ("gauss", 40.0, 127))
    want = oracle_mod.xcorr(x, ns, npol)
    st = X.Stream(ns, npol, F, chunk, "ci8", acc)
    out = st.begin()
    for c in range(nchunk):
        st.push(torch.from_numpy(np.ascontiguousarray(x[c * chunk:(c + 1) * chunk])).pin_memory())
    assert st.end() == chunk * nchunk
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), want, f"chan-stream/{acc}")
    st.close()
