"""GPU parity of the streaming integration (Algorithm 1): chunks copied from pinned host
memory while earlier chunks are correlated; the totals equal the oracle over the whole
integration (time linearity, exact in integers)."""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, device, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("acc", ["i8", "f16", "f32", "f8"])
def test_stream_matches_oracle(oracle_mod, acc):
    import torch

    from paper_1107_4264_amd import xcorr as X

    device()
    ns, npol, F, chunk, nchunk = 36, 2, 5, 96, 5
    dist = ("uniform", -16, 16) if acc == "f8" else ("gauss", 60.0, 127)
    x = synth.voltages_np(4242, chunk * nchunk, F, ns * npol, dist)
    want = oracle_mod.xcorr(x, ns, npol)
    say("stream", acc)
    st = X.Stream(ns, npol, F, chunk, "ci8", acc, max_abs=16 if acc == "f8" else None)
    chunks = [torch.from_numpy(np.ascontiguousarray(x[c * chunk:(c + 1) * chunk])).pin_memory()
              for c in range(nchunk)]
    out = st.begin()
    for c in range(nchunk):
        st.push(chunks[c])
    assert st.end() == chunk * nchunk
    torch.cuda.synchronize()
    assert np.array_equal(as_exact_int(out.cpu().numpy()), want)
    # a second integration over the chunks in reverse order gives the same totals
    out2 = st.begin()
    for c in reversed(range(nchunk)):
        st.push(chunks[c])
    st.end()
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    st.close()


def test_stream_windows_within_chunk(oracle_mod):
    """Chunks longer than an exact window (fp32 accumulators at the default 8-bit bound)."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    ns, npol, F, chunk, nchunk = 6, 2, 2, 1200, 3
    x = synth.voltages_np(99, chunk * nchunk, F, ns * npol, ("gauss", 100.0, 127))
    want = oracle_mod.xcorr(x, ns, npol)
    st = X.Stream(ns, npol, F, chunk, "ci8", "f16")
    out = st.begin()
    for c in range(nchunk):
        st.push(torch.from_numpy(np.ascontiguousarray(x[c * chunk:(c + 1) * chunk])).pin_memory())
    st.end()
    torch.cuda.synchronize()
    assert np.array_equal(as_exact_int(out.cpu().numpy()), want)
    st.close()


@pytest.mark.parametrize("acc", ["i8", "f16"])
def test_stream_graph_replays(oracle_mod, acc):
    """A whole integration captured once as a HIP graph: each replay re-reads the pinned
    chunks and recomputes the totals; replays are interleaved with eager work and host
    synchronisation, and every replay is checked (the zero fill is a kernel, not a memset
    node)."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    dev = device()
    ns, npol, F, chunk, nchunk = 128, 2, 3, 64, 4
    st = X.Stream(ns, npol, F, chunk, "ci8", acc)
    chunks = [torch.empty((chunk, F, ns * npol, 2), dtype=torch.int8).pin_memory() for _ in range(nchunk)]
    out = st.empty_out(dev)
    g = st.capture(chunks, out)
    for rep in range(3):
        x = synth.voltages_np(5150 + rep, chunk * nchunk, F, ns * npol, ("gauss", 40.0, 127))
        for c in range(nchunk):
            chunks[c].copy_(torch.from_numpy(np.ascontiguousarray(x[c * chunk:(c + 1) * chunk])))
        # some eager work on the device between replays
        junk = torch.randn(1 << 20, device=dev)
        junk.mul_(2.0)
        torch.cuda.synchronize()
        say("graph replay", acc, rep)
        g.launch()
        torch.cuda.synchronize()
        assert np.array_equal(as_exact_int(out.cpu().numpy()), oracle_mod.xcorr(x, ns, npol)), rep
    # the same stream object still runs eagerly afterwards
    x = synth.voltages_np(5160, chunk * nchunk, F, ns * npol, ("gauss", 40.0, 127))
    out2 = st.begin()
    for c in range(nchunk):
        st.push(torch.from_numpy(np.ascontiguousarray(x[c * chunk:(c + 1) * chunk])).pin_memory())
    st.end()
    torch.cuda.synchronize()
    assert np.array_equal(as_exact_int(out2.cpu().numpy()), oracle_mod.xcorr(x, ns, npol))
    g.close()
    st.close()
