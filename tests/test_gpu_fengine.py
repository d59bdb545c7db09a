"""GPU F-engine and corner turn against the F-engine oracle, and the whole FX chain: the
transform itself (fp32 spectra within the normwise rounding bound of an fp32 FFT), the
requantised 8-bit output (equal to the oracle's except where the exact value lies within
that bound of a rounding boundary, and there off by at most one, on at most 0.1 % of the
components), and the X-engine run on
the F-engine's output against the X-engine oracle on the same samples (bit for bit)."""

from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import fengine as FE
from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, device, say

pytestmark = pytest.mark.gpu

U32 = 2.0**-24


def _volts(seed, nin, nsamp, sigma=20.0):
    v = synth.voltages_np(seed, nsamp, 1, nin, ("gauss", sigma, 127))  # [nsamp][1][nin][2]
    return np.ascontiguousarray(np.transpose(v[:, 0], (1, 0, 2)))      # [nin][nsamp][2]


def _gain(nchan):
    return 0.5 / math.sqrt(nchan)


def _run(x, ns, npol, nchan, nframes, gain, spectra):
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    e = X.FEngine(ns, npol, nchan, nframes, gain)
    out = e.run(torch.from_numpy(x).to(dev), spectra=spectra)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    e.close()
    return res


def _bound(want, nchan):
    """Normwise bound per (frame, input) of an fp32 radix-2 FFT: 5 log2(F) u ||X||_2."""
    return 5.0 * math.log2(nchan) * U32 * np.sqrt(np.sum(np.abs(want) ** 2, axis=1, keepdims=True))


SHAPES = [
    # (nstation, npol, nchan, nframes)
    (16, 2, 64, 5),
    (37, 1, 128, 3),      # 37 inputs: a partial input group, odd rows
    (50, 2, 256, 4),      # 100 inputs
    (128, 2, 1024, 3),    # the benchmark's 256 inputs x 1024 channels
    (9, 2, 2048, 2),
    (33, 1, 512, 1),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_spectra_within_fp32_bound(shape):
    ns, npol, nchan, nframes = shape
    nin = ns * npol
    x = _volts(7000 + nchan + nin, nin, nchan * nframes)
    gain = _gain(nchan)
    want = FE.channelise(x, nchan, gain)                       # [t][k][i] complex128
    got = _run(x, ns, npol, nchan, nframes, gain, True)
    gc = got[..., 0].astype(np.float64) + 1j * got[..., 1]
    err = np.sqrt(np.sum(np.abs(gc - want) ** 2, axis=1, keepdims=True))
    bound = _bound(want, nchan)
    ratio = float(np.max(err / bound))
    say("spectra", shape, "max normwise error / bound", f"{ratio:.3f}")
    assert ratio <= 1.0


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_requantised_matches_oracle(shape):
    ns, npol, nchan, nframes = shape
    nin = ns * npol
    x = _volts(7100 + nchan + nin, nin, nchan * nframes)
    gain = _gain(nchan)
    spec = FE.channelise(x, nchan, gain)
    want = FE.requantise(spec)
    got = _run(x, ns, npol, nchan, nframes, gain, False)
    assert got.shape == want.shape and got.dtype == np.int8
    # components whose exact value lies within the fp32 error bound of a rounding boundary
    margin = np.broadcast_to(_bound(spec, nchan), spec.shape)
    near = np.zeros(want.shape, dtype=bool)
    for c, part in enumerate((spec.real, spec.imag)):
        frac = np.abs(np.abs(part) - np.floor(np.abs(part)) - 0.5)
        near[..., c] = (frac <= margin) & (np.abs(part) < 127.5)
    diff = got.astype(np.int16) - want
    say("requantised", shape, "ambiguous components", int(near.sum()), "differing", int((diff != 0).sum()))
    assert np.all(diff[~near] == 0)
    assert np.all(np.abs(diff[near]) <= 1)
    # the bound is a worst case: at least 90 % of the components are checked exactly, and
    # the fp32 / fp64 roundings part on at most 0.1 % of them
    assert near.sum() <= want.size // 10
    assert (diff != 0).sum() <= max(2, want.size // 1000)


@pytest.mark.parametrize("acc", ["i8", "f16"])
def test_fx_chain(oracle_mod, acc):
    """F-engine output straight into the X-engine: the visibilities equal the X-engine
    oracle's on the same requantised samples."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    ns, npol, nchan, nframes = 24, 2, 256, 40
    nin = ns * npol
    x = _volts(7200, nin, nchan * nframes)
    e = X.FEngine(ns, npol, nchan, nframes, _gain(nchan))
    samples = e.run(torch.from_numpy(x).to(dev))
    c = X.Correlator(ns, npol, nchan, nframes, "ci8", acc)
    vis = c.run(samples.view(torch.int8))
    torch.cuda.synchronize()
    s = samples.cpu().numpy()                                  # [t][k][i][2]
    want = oracle_mod.xcorr(s, ns, npol)
    assert np.array_equal(as_exact_int(vis.cpu().numpy()), want)
    e.close()
    c.close()


def test_fengine_argument_checks():
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    for nchan in (48, 96, 4096, 32):
        with pytest.raises(X.XcorrError):
            X.FEngine(4, 2, nchan, 2, 0.1)
    with pytest.raises(X.XcorrError):
        X.FEngine(4, 2, 64, 2, 0.0)
    e = X.FEngine(4, 2, 64, 2, 0.1)
    buf = torch.zeros(4 * 2 * 64 * 2 + 2, dtype=torch.uint8, device=dev)
    out = e.empty_out(dev)
    with pytest.raises(X.XcorrError) as ei:
        X.xcorr_fengine_run(e.e, buf.data_ptr() + 2, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert ei.value.code == X.ERR_INVALID_ARG
    e.close()
    z = X.FEngine(4, 2, 64, 0, 0.1)  # no frames: nothing to do
    X.xcorr_fengine_run(z.e, 0, 0, 0)
    z.close()
