"""GPU parity at the stated sizes of the benchmark workloads, on sampled channels the oracle
computes one by one: 256 inputs x 1024 channels x 1000 8-bit samples (FP32 CMAC, fp16 and
int8 matrix cores) and 1024 inputs x 256 channels x 4096 4-bit samples (int8 and fp8
matrix cores on super-tiles, fp6 on 128-tiles).  Inputs come from the same seeded generator as the
benchmark, evaluated on the device for the GPU run and on the host for the sampled
channels."""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, device, say

pytestmark = pytest.mark.gpu


def _sampled(oracle_mod, out, want, chans, label):
    got = as_exact_int(out[chans].cpu().numpy())
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        say(label, "MISMATCH count", len(bad), "first", bad[:5].tolist())
    assert np.array_equal(got, want), label


def test_n256_ci8_full_size(oracle_mod):
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    ns, npol, F, T = 128, 2, 1024, 1000
    nin = ns * npol
    dist = ("gauss", 3.0, 127)
    seed = synth.SEED_BASE + 1
    x = synth.voltages_torch(seed, T, F, nin, dist, dev)
    torch.cuda.synchronize()
    m = int(x.abs().max().item())
    chans = [0, 333, 700, F - 1]
    want = oracle_mod.xcorr(synth.voltages_np(seed, T, F, nin, dist, chans=chans), ns, npol)
    for acc in ("f32", "f16", "i8"):
        say("full size 256 inputs", acc)
        c = X.Correlator(ns, npol, F, T, "ci8", acc, max_abs=m)
        out = c.run(x)
        torch.cuda.synchronize()
        _sampled(oracle_mod, out, want, chans, f"n256/{acc}")
        c.close()
        del out


def test_n1024_ci4_full_size(oracle_mod):
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    ns, npol, F, T = 512, 2, 256, 4096
    nin = ns * npol
    dist = ("uniform", -8, 7)
    seed = synth.SEED_BASE + 2
    v = synth.voltages_torch(seed, T, F, nin, dist, dev)
    x = synth.pack_ci4_torch(v)
    del v
    torch.cuda.synchronize()
    chans = [0, 77, 190, F - 1]
    want = oracle_mod.xcorr(synth.pack_ci4(synth.voltages_np(seed, T, F, nin, dist, chans=chans)), ns, npol,
                            fmt=oracle_mod.CI4)
    for acc in ("i8", "f8", "f6"):
        say("full size 1024 inputs", acc)
        c = X.Correlator(ns, npol, F, T, "ci4", acc)
        assert c.tile == 512
        out = c.run(x)
        torch.cuda.synchronize()
        _sampled(oracle_mod, out, want, chans, f"n1024/{acc}")
        c.close()
        del out
