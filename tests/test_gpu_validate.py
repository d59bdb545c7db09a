"""GPU tests of the optional range check (the exactness conditions of Sec. 2.3; on the
int8 path a -128 component would overflow when the imaginary product negates it).

The count of out-of-range components is compared with numpy's count on the same seeded
input; with validation on, a run over such input is refused with XCORR_ERR_RANGE and leaves
the output untouched, and a run over clean input gives the oracle's visibilities.
"""

from __future__ import annotations

import ctypes

import numpy as np
import pytest

from oracle import CI4, CI8
from oracle import xcorr as oracle_xcorr
from tests.gpu_util import as_exact_int, device, say

pytestmark = pytest.mark.gpu


def _count_ci8(x, m):
    v = x.astype(np.int32)
    return int(np.count_nonzero((v > m) | (v < -m)))


def _count_ci4(x, m):
    hi = (x >> 4).astype(np.int32)
    lo = (x & 15).astype(np.int32)
    hi = hi - 16 * (hi >= 8)
    lo = lo - 16 * (lo >= 8)
    return int(np.count_nonzero((hi > m) | (hi < -m)) + np.count_nonzero((lo > m) | (lo < -m)))


# (stations, pol, channels, samples): one with an input size that is not a multiple of 16
# bytes, one large enough for many workgroups of the check
SHAPES = [(5, 2, 3, 7), (64, 2, 33, 100)]


@pytest.mark.parametrize("shape", SHAPES)
def test_int8_path_counts_minus_128(shape):
    import torch

    from paper_1107_4264_amd import xcorr as X

    ns, npol, nchan, ntime = shape
    nin = ns * npol
    rng = np.random.default_rng(1234 + ns)
    x = rng.integers(-127, 128, size=(ntime, nchan, nin, 2), dtype=np.int64).astype(np.int8)
    dev = device()
    c = X.Correlator(ns, npol, nchan, ntime, "ci8", "i8")
    assert c.count_out_of_range(torch.from_numpy(x).to(dev)) == 0
    flat = x.reshape(-1)
    pos = np.unique(np.concatenate([rng.integers(0, flat.size, size=5), [0, flat.size - 1]]))
    flat[pos] = -128
    want = _count_ci8(x, 127)
    assert want == len(pos)
    xt = torch.from_numpy(x).to(dev)
    got = c.count_out_of_range(xt)
    say("int8 -128 count", shape, got, "want", want)
    assert got == want
    # with validation on the run is refused and the output keeps its contents
    cv = X.Correlator(ns, npol, nchan, ntime, "ci8", "i8", validate=True)
    out = cv.empty_out(dev)
    out.fill_(7)
    with pytest.raises(X.XcorrError) as ei:
        cv.run(xt, out)
    assert ei.value.code == X.ERR_RANGE
    torch.cuda.synchronize()
    assert bool((out == 7).all())
    # clean input: the validated run equals the oracle
    flat[pos] = 5
    xt = torch.from_numpy(x).to(dev)
    got_out = cv.run(xt, out)
    torch.cuda.synchronize()
    want_out = oracle_xcorr(x, ns, npol, CI8)
    assert np.array_equal(as_exact_int(got_out.cpu().numpy()), want_out)


def test_declared_bound_on_fp16_path():
    import torch

    from paper_1107_4264_amd import xcorr as X

    ns, npol, nchan, ntime = 16, 2, 5, 64
    rng = np.random.default_rng(99)
    x = rng.integers(-18, 19, size=(ntime, nchan, ns * npol, 2), dtype=np.int64).astype(np.int8)
    flat = x.reshape(-1)
    flat[[3, 77, 1000]] = [19, -19, -128]
    flat[[5, 6]] = [18, -18]
    c = X.Correlator(ns, npol, nchan, ntime, "ci8", "f16", max_abs=18)
    got = c.count_out_of_range(torch.from_numpy(x).to(device()))
    assert got == _count_ci8(x, 18) == 3
    # without a declared bound the fp16 path holds every 8-bit value
    c2 = X.Correlator(ns, npol, nchan, ntime, "ci8", "f16")
    assert c2.count_out_of_range(torch.from_numpy(x).to(device())) == 0


def test_ci4_declared_bound():
    import torch

    from paper_1107_4264_amd import xcorr as X

    ns, npol, nchan, ntime = 9, 2, 4, 65
    rng = np.random.default_rng(7)
    re = rng.integers(-7, 8, size=(ntime, nchan, ns * npol))
    im = rng.integers(-7, 8, size=(ntime, nchan, ns * npol))
    re.reshape(-1)[[0, 10]] = -8
    im.reshape(-1)[[11, re.size - 1]] = -8
    x = (((re & 15) << 4) | (im & 15)).astype(np.uint8)
    dev = device()
    c7 = X.Correlator(ns, npol, nchan, ntime, "ci4", "i8", max_abs=7)
    assert c7.count_out_of_range(torch.from_numpy(x).to(dev)) == _count_ci4(x, 7) == 4
    c8 = X.Correlator(ns, npol, nchan, ntime, "ci4", "i8")
    assert c8.count_out_of_range(torch.from_numpy(x).to(dev)) == 0
    cv = X.Correlator(ns, npol, nchan, ntime, "ci4", "i8", validate=True)
    out = cv.run(torch.from_numpy(x).to(dev))
    torch.cuda.synchronize()
    assert np.array_equal(as_exact_int(out.cpu().numpy()), oracle_xcorr(x, ns, npol, CI4))


@pytest.mark.parametrize("offset", [1, 3, 8, 15])
def test_unaligned_input_pointer(offset):
    """The check reads any byte alignment: bytes before the first 16-byte boundary, the
    aligned body and the tail."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    ns, npol, nchan, ntime = 3, 2, 5, 11
    nbytes = ntime * nchan * ns * npol * 2
    rng = np.random.default_rng(offset)
    buf = rng.integers(-127, 128, size=nbytes + 32, dtype=np.int64).astype(np.int8)
    body = buf[offset:offset + nbytes]
    body[[0, 1, nbytes // 2, nbytes - 1]] = -128
    buf[offset - 1] = -128            # just before the input: not counted
    buf[offset + nbytes] = -128       # just after it: not counted
    dev = device()
    bt = torch.from_numpy(buf).to(dev)
    c = X.Correlator(ns, npol, nchan, ntime, "ci8", "i8")
    got = X.xcorr_validate(c.h, ctypes.c_void_p(bt.data_ptr() + offset), None)
    say("unaligned", offset, got)
    assert got == _count_ci8(body, 127) == 4
