"""Helpers shared by the GPU tests: run the HIP X-engine through the C ABI and compare with
the oracle on the same seeded inputs."""

from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


# Largest sample component the low-precision operand types hold exactly (8-bit samples on
# these paths need the bound declared).
LOWBIT = {"f8": 16, "f6": 8}


def low_dist(acc, default):
    """Sample distribution for 8-bit samples on path acc: uniform within the operand type's
    exact range on the fp8 / fp6 paths, `default` otherwise."""
    m = LOWBIT.get(acc)
    return ("uniform", -m, m) if m else default


def low_max_abs(acc):
    return LOWBIT.get(acc)


def device():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a GPU")
    return torch.device("cuda:0")


def run_xeng(x_np, nstation, npol, in_dtype, acc, max_abs=None, nchan=None, tile=None):
    """Copy x to the device, run one job (tile None: the automatic kernel shape), return
    (numpy output, out_type)."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    xt = torch.from_numpy(np.ascontiguousarray(x_np)).to(dev)
    ntime = x_np.shape[0]
    nchan = x_np.shape[1] if nchan is None else nchan
    c = X.Correlator(nstation, npol, nchan, ntime, in_dtype, acc, max_abs=max_abs, tile=tile)
    if tile is not None:
        assert c.tile == tile
    out = c.run(xt)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    ot = c.out_type
    c.close()
    return res, ot


def as_exact_int(o: np.ndarray) -> np.ndarray:
    """Integer-valued output of any type -> int64 (asserting the floats are integers)."""
    if o.dtype.kind == "f":
        r = np.rint(o)
        assert np.array_equal(r, o), "float output is not integer valued"
        return r.astype(np.int64)
    return o.astype(np.int64)
