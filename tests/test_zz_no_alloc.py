"""The batch entry point that allocates nothing (xcorr_batch_run_noalloc), through the C ABI,
against the batch entry point that allocates its work list (xcorr_batch_create / run): the
same visibilities, bit for bit, on two calls in a row (the second smaller, so the fixed
workspace holds the previous call's table and counts), on the FP32 CMAC, int8 and fp16
paths, with jobs on the tiled kernel (several windows included), the whole-channel kernel
and the super-tiles; one job also against the oracle."""

from __future__ import annotations

import ctypes

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, device, say

pytestmark = pytest.mark.gpu

FIRST = [
    # (nstation, npol, nchan, ntime)
    (3, 2, 4, 37),
    (25, 2, 11, 130),   # nin 50: word loads
    (100, 2, 5, 65),    # nin 200: ragged 128-tiles
    (17, 1, 3, 64),     # odd nin: byte loads
    (40, 2, 9, 1100),   # several fp32 windows at the default bound
    (128, 2, 3, 96),    # nin 256: whole channel on the int8 / fp16 paths
    (256, 2, 2, 40),    # nin 512: super-tiles on the int8 path
    (12, 2, 3, 0),      # no samples
]
SECOND = [
    (9, 2, 2, 50),
    (30, 2, 3, 70),
]


def _inputs(jobs, seed, dev):
    import torch

    xs = [synth.voltages_np(seed + 16 * k, T, F, ns * npol, ("gauss", 50.0, 127))
          for k, (ns, npol, F, T) in enumerate(jobs)]
    return xs, [torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in xs]


def _noalloc(jobs, acc, xt, outs):
    import torch

    from paper_1107_4264_amd import xcorr as X

    X.xcorr_batch_run_noalloc(jobs, X.IN_CI8, X.ACC_NAMES[acc], 0, [x.data_ptr() for x in xt],
                              [o.data_ptr() for o in outs], ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("acc", ["f32", "i8", "f16"])
def test_noalloc_matches_batch(oracle_mod, acc):
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    for call, (jobs, seed) in enumerate(((FIRST, 4100), (SECOND, 4200))):
        xs, xt = _inputs(jobs, seed, dev)
        b = X.Batch(jobs, "ci8", acc)
        want = b.run(xt)
        got = [torch.full_like(o, 7) for o in want]  # stale values must be overwritten
        say("noalloc", acc, "call", call, "jobs", len(jobs))
        _noalloc(jobs, acc, xt, got)
        torch.cuda.synchronize()
        for k, (g, w) in enumerate(zip(got, want)):
            assert g.dtype == w.dtype and torch.equal(g, w), f"call {call} job {k} {jobs[k]}"
        ns, npol, F, T = jobs[1]
        assert np.array_equal(as_exact_int(got[1].cpu().numpy()), oracle_mod.xcorr(xs[1], ns, npol))
        b.close()


def test_noalloc_rejects_too_many_jobs():
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    n = 257
    jobs = [(2, 1, 1, 4)] * n
    x = torch.zeros(4 * 2 * 2, dtype=torch.int8, device=dev)
    o = torch.zeros(64, dtype=torch.float32, device=dev)
    with pytest.raises(X.XcorrError) as e:
        X.xcorr_batch_run_noalloc(jobs, X.IN_CI8, X.ACC_F32_CMAC, 0, [x.data_ptr()] * n, [o.data_ptr()] * n,
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert e.value.code == X.ERR_INVALID_ARG
    assert "256" in X.last_error()
