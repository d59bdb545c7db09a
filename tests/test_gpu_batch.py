"""GPU parity of the persistent batched launch: uneven jobs in one launch against the oracle
(and against the single-job launch of the same job)."""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, device, low_dist, low_max_abs, run_xeng, say

pytestmark = pytest.mark.gpu

JOBS = [
    # (nstation, npol, nchan, ntime)
    (3, 2, 4, 37),
    (25, 2, 3, 130),    # nin 50: word loads
    (64, 2, 2, 200),    # nin 128: one tile
    (100, 2, 5, 65),    # nin 200: ragged 128-tiles
    (17, 1, 3, 64),     # odd nin: byte loads
    (40, 2, 9, 1100),   # several fp32 windows at the default bound
]


@pytest.mark.parametrize("acc", ["f32", "i8", "f16", "f8", "f32m", "f6"])
def test_batch_matches_oracle(oracle_mod, acc):
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    dist = low_dist(acc, ("gauss", 50.0, 127))
    xs, wants = [], []
    for k, (ns, npol, F, T) in enumerate(JOBS):
        x = synth.voltages_np(synth.SEED_BASE + 3 + 16 * k, T, F, ns * npol, dist)
        xs.append(x)
        wants.append(oracle_mod.xcorr(x, ns, npol))
    say("batch", acc, "jobs", len(JOBS))
    b = X.Batch(JOBS, "ci8", acc, max_abs=low_max_abs(acc))
    assert X.xcorr_batch_items(b.b) > 0
    outs = b.run([torch.from_numpy(x).to(dev) for x in xs])
    torch.cuda.synchronize()
    for k, (o, want) in enumerate(zip(outs, wants)):
        got = as_exact_int(o.cpu().numpy())
        assert np.array_equal(got, want), f"job {k} {JOBS[k]}"
    # same bits as launching each job alone
    for k, (ns, npol, F, T) in enumerate(JOBS[:3]):
        single, _ = run_xeng(xs[k], ns, npol, "ci8", acc, max_abs=low_max_abs(acc))
        assert np.array_equal(single, outs[k].cpu().numpy())
    # run twice: same bits (counters and zero fills are reset per run)
    outs2 = b.run([torch.from_numpy(x).to(dev) for x in xs])
    torch.cuda.synchronize()
    for o1, o2 in zip(outs, outs2):
        assert torch.equal(o1, o2)
    b.close()


def test_batch_ci4(oracle_mod):
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    jobs = [(16, 2, 3, 50), (70, 2, 2, 129), (9, 1, 4, 33)]
    xs, wants = [], []
    for k, (ns, npol, F, T) in enumerate(jobs):
        v = synth.voltages_np(777 + k, T, F, ns * npol, ("uniform", -8, 7))
        p = synth.pack_ci4(v)
        xs.append(p)
        wants.append(oracle_mod.xcorr(p, ns, npol, fmt=oracle_mod.CI4))
    for acc in ["i8", "f16", "f8", "f32m", "f6"]:
        say("batch ci4", acc)
        b = X.Batch(jobs, "ci4", acc)
        outs = b.run([torch.from_numpy(x).to(dev) for x in xs])
        torch.cuda.synchronize()
        for k, (o, want) in enumerate(zip(outs, wants)):
            assert np.array_equal(as_exact_int(o.cpu().numpy()), want), f"{acc} job {k}"
        b.close()


def test_batch_mixed_kernels(oracle_mod):
    """One batch whose jobs run on three kernels: a 512-input job (super-tiles), a
    256-input job (whole channel) and small jobs (the persistent tiled launch), for 8-bit
    samples on the int8 path and 4-bit samples on the int8 and fp8 paths."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    for fmt, accs in (("ci8", ["i8"]), ("ci4", ["i8", "f8"])):
        jobs = [(256, 2, 2, 70), (128, 2, 3, 50), (21, 2, 2, 40), (5, 1, 3, 9)]
        xs, wants = [], []
        for k, (ns, npol, F, T) in enumerate(jobs):
            if fmt == "ci8":
                x = synth.voltages_np(880 + k, T, F, ns * npol, ("gauss", 30.0, 127))
                xs.append(x)
                wants.append(oracle_mod.xcorr(x, ns, npol))
            else:
                p = synth.pack_ci4(synth.voltages_np(890 + k, T, F, ns * npol, ("uniform", -8, 7)))
                xs.append(p)
                wants.append(oracle_mod.xcorr(p, ns, npol, fmt=oracle_mod.CI4))
        for acc in accs:
            say("batch mixed", fmt, acc)
            b = X.Batch(jobs, fmt, acc)
            outs = b.run([torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in xs])
            torch.cuda.synchronize()
            for k, (o, want) in enumerate(zip(outs, wants)):
                assert np.array_equal(as_exact_int(o.cpu().numpy()), want), f"{fmt} {acc} job {k}"
            b.close()
