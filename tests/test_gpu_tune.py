"""GPU autotuner: every candidate shape is timed on the device, the result is bit-exact,
and the tuned shape is recorded and reused by new handles of the same job shape."""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, device, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("acc", ["f16", "i8"])
def test_autotune_picks_a_shape_and_keeps_bits(oracle_mod, acc, tmp_path):
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
        # every allowed shape was timed: the whole-channel kernel's four variants and the
        # tiles of 128 and 64, each staged in LDS and through the caches
        res = X.xcorr_autotune_results(c.h)
        shapes = {(r["tile"], r["staging"], r["variant"]) for r in res}
        say("autotune", acc, "timed", sorted(shapes))
        assert {(256, 0, v) for v in range(4)} <= shapes
        assert {(128, 0, 0), (128, 1, 0), (64, 0, 0), (64, 1, 0)} <= shapes
        assert all(r["us"] > 0 for r in res)
        best = min(res, key=lambda r: r["us"])
        assert (best["tile"], best["staging"], best["variant"]) == (c.tile, c.staging, c.variant)
        # recorded under the job's class on this device's architecture (the default bound)
        assert X.xcorr_autotune_lookup(ns, npol, F, T, X.IN_CI8, X.ACC_NAMES[acc], 0, full=True) == \
            (c.tile, c.staging, c.variant)
        assert X.xcorr_autotune_lookup(ns, npol, F, T, X.IN_CI8, X.ACC_NAMES[acc], 0, arch="gfx950") == tile
        # the class covers other channel / sample counts in the same power-of-two buckets
        assert X.xcorr_autotune_lookup(ns, npol, F + 20, T + 100, X.IN_CI8, X.ACC_NAMES[acc], 0) == tile
        path = tmp_path / "tuned.jsonl"
        assert X.xcorr_autotune_save(str(path)) == 1
        assert '"arch": "gfx950"' in path.read_text()
        c2 = X.Correlator(ns, npol, F, T, "ci8", acc)
        assert (c2.tile, c2.staging, c2.variant) == (c.tile, c.staging, c.variant)
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
        shapes = {(r["tile"], r["staging"], r["variant"]) for r in X.xcorr_autotune_results(c.h)}
        assert {(512, 0, 0), (512, 0, 1), (128, 1, 0)} <= shapes
        want = oracle_mod.xcorr(packed, ns, npol, fmt=oracle_mod.CI4)
        assert np.array_equal(as_exact_int(out.cpu().numpy()), want)
        c.close()
    finally:
        X.xcorr_autotune_clear()
