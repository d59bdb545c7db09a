"""GPU autotuner: every candidate shape is timed on the device, the result is bit-exact,
and the tuned shape is recorded and reused by new handles of the same job shape."""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, device, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("acc", ["f16", "i8"])
def test_autotune_picks_a_shape_and_keeps_bits(oracle_mod, acc):
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    ns, npol, F, T = 128, 2, 40, 300
    x = synth.voltages_np(synth.SEED_BASE + 60, T, F, ns * npol, ("gauss", 30.0, 127))
    xt = torch.from_numpy(x).to(dev)
    X.xcorr_autotune_clear()
    try:
        c = X.Correlator(ns, npol, F, T, "ci8", acc)
        out = c.empty_out(dev)
        tile = c.autotune(xt, out, reps=2)
        torch.cuda.synchronize()
        say("autotune", acc, "tile", tile)
        assert tile in (64, 128, 256) and c.tile == tile
        want = oracle_mod.xcorr(x, ns, npol)
        assert np.array_equal(as_exact_int(out.cpu().numpy()), want)
        # recorded under the job shape (the handle's bound is the default one here)
        assert X.xcorr_autotune_lookup(ns, npol, F, T, X.IN_CI8, X.ACC_NAMES[acc], 0) == tile
        c2 = X.Correlator(ns, npol, F, T, "ci8", acc)
        assert c2.tile == tile
        got = c2.run(xt)
        torch.cuda.synchronize()
        assert np.array_equal(as_exact_int(got.cpu().numpy()), want)
        c.close()
        c2.close()
    finally:
        X.xcorr_autotune_clear()


@pytest.mark.parametrize("acc", ["i8", "f8"])
def test_autotune_includes_super_tiles(oracle_mod, acc):
    """A 4-bit job of 512 inputs: the candidates include super-tiles (512), 128 and 64;
    whichever wins, the visibilities are the oracle's."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    ns, npol, F, T = 256, 2, 6, 200
    packed = synth.pack_ci4(synth.voltages_np(synth.SEED_BASE + 61, T, F, ns * npol, ("uniform", -8, 7)))
    xt = torch.from_numpy(packed).to(dev)
    X.xcorr_autotune_clear()
    try:
        c = X.Correlator(ns, npol, F, T, "ci4", acc)
        assert c.tile == 512
        out = c.empty_out(dev)
        tile = c.autotune(xt, out, reps=2)
        torch.cuda.synchronize()
        say("autotune ci4", acc, "tile", tile)
        assert tile in (64, 128, 512) and c.tile == tile
        want = oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4)
        assert np.array_equal(as_exact_int(out.cpu().numpy()), want)
        c.close()
    finally:
        X.xcorr_autotune_clear()
