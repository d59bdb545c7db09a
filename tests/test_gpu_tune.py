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
