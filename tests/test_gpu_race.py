"""Race tests of the copy / compute ordering (Algorithm 1 synchronises the host with the
copies of every iteration; the library orders copies, kernels and buffer reuse with events):
the same integer totals, bit for bit, with seeded random host delays that shift the host
against the copies and kernels, and with the runtime serialising every kernel and copy
(AMD_SERIALIZE_KERNEL / AMD_SERIALIZE_COPY, in a child process).  A missing wait shows as
totals that differ between these runs or from the oracle."""

from __future__ import annotations

import os
import subprocess
import sys

import numpy as np
import pytest

from tests import race_workload as W
from tests.gpu_util import as_exact_int, device, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _oracle_results(oracle_mod):
    xs, xb, x1 = W.inputs()
    ns, npol = W.STREAM_SHAPE[:2]
    want = {"stream": oracle_mod.xcorr(xs, ns, npol)}
    for k, (s, p, f, t) in enumerate(W.BATCH_JOBS):
        want[f"batch{k}"] = oracle_mod.xcorr(xb[k], s, p)
    want["single"] = oracle_mod.xcorr(x1, W.SINGLE[0], W.SINGLE[1])
    return want


def _same(got, want, label):
    assert sorted(got) == sorted(want)
    for k in want:
        assert np.array_equal(as_exact_int(got[k]), want[k]), f"{label}: {k}"


def test_random_host_delays(oracle_mod):
    device()
    want = _oracle_results(oracle_mod)
    for seed in (11, 12, 13):
        say("race workload, host delay seed", seed)
        _same(W.run(seed), want, f"delays seed {seed}")


def test_serialised_runtime(oracle_mod, tmp_path):
    device()
    want = _oracle_results(oracle_mod)
    out = str(tmp_path / "serial.npz")
    env = dict(os.environ, AMD_SERIALIZE_KERNEL="3", AMD_SERIALIZE_COPY="3")
    say("race workload in a child process with serialised kernels and copies")
    r = subprocess.run([sys.executable, "-m", "tests.race_workload", out], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    got = dict(np.load(out))
    _same(got, want, "serialised")
    # and the same bits without serialisation, in this process
    _same(W.run(None), want, "unserialised")
