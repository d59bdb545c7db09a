"""GPU parity of the streaming integration (Algorithm 1): chunks copied from pinned host
memory while earlier chunks are correlated; the totals equal the oracle over the whole
integration (time linearity, exact in integers)."""

from __future__ import annotations

import numpy as np
import pytest

from paper_1107_4264_amd import synth
from tests.gpu_util import as_exact_int, device, low_dist, low_max_abs, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("acc", ["i8", "f16", "f32", "f8", "f32m", "f6"])
def test_stream_matches_oracle(oracle_mod, acc):
    import torch

    from paper_1107_4264_amd import xcorr as X

    device()
    ns, npol, F, chunk, nchunk = 36, 2, 5, 96, 5
    dist = low_dist(acc, ("gauss", 60.0, 127))
    x = synth.voltages_np(4242, chunk * nchunk, F, ns * npol, dist)
    want = oracle_mod.xcorr(x, ns, npol)
    say("stream", acc)
    st = X.Stream(ns, npol, F, chunk, "ci8", acc, max_abs=low_max_abs(acc))
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


def _release_run(oracle_mod, delays):
    """Pushes from a pool of three pinned buffers, each refilled with its next chunk right
    after the push that releases it (push p releases chunk p - 2, so buffer p % 3 is free
    once push p - 1 has returned).  Optional host delays (seeded) between the steps shift
    the host against the copies and kernels."""
    import time

    import torch

    from paper_1107_4264_amd import xcorr as X

    device()
    ns, npol, F, chunk, nchunk = 256, 2, 64, 256, 9
    nin = ns * npol
    x = synth.voltages_np(synth.SEED_BASE + 97, chunk * nchunk, F, nin, ("gauss", 30.0, 127))
    want = oracle_mod.xcorr(x, ns, npol, chans=[0, F // 2, F - 1])
    bufs = [torch.empty((chunk, F, nin, 2), dtype=torch.int8).pin_memory() for _ in range(3)]
    src = [torch.from_numpy(np.ascontiguousarray(x[c * chunk:(c + 1) * chunk])) for c in range(nchunk)]
    rng = np.random.default_rng(5)
    st = X.Stream(ns, npol, F, chunk, "ci8", "i8")
    out = st.empty_out()
    X.xcorr_stream_begin(st.s, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    bufs[0].copy_(src[0])
    bufs[1].copy_(src[1])
    for p in range(nchunk):
        if p >= 2:
            # chunk p - 3 (buffer p % 3) was released when push p - 1 returned
            if delays:
                time.sleep(float(rng.uniform(0.0, 0.004)))
            bufs[p % 3].copy_(src[p])
        if delays:
            time.sleep(float(rng.uniform(0.0, 0.004)))
        X.xcorr_stream_push(st.s, bufs[p % 3].data_ptr(), torch.cuda.current_stream().cuda_stream)
    assert X.xcorr_stream_end(st.s, torch.cuda.current_stream().cuda_stream) == chunk * nchunk
    torch.cuda.synchronize()
    got = out[[0, F // 2, F - 1]].cpu().numpy()
    assert np.array_equal(as_exact_int(got), want)
    st.close()


def test_stream_chunk_reuse_at_release_point(oracle_mod):
    say("stream release point")
    _release_run(oracle_mod, delays=False)


def test_stream_chunk_reuse_random_delays(oracle_mod):
    say("stream release point, random host delays")
    _release_run(oracle_mod, delays=True)
