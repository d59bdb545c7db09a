"""Workload of the race tests: a streaming integration whose pinned chunks are refilled at
the documented release point, a batch of uneven jobs with eager work on a second stream
between its launches, and a single job, each optionally with seeded random host delays.

Run as a program (``python -m tests.race_workload OUT.npz``) it writes the results, so a
test can run it in a child process with the runtime's serialisation switches set and
compare bit for bit.  No part of the library's arithmetic is here.
"""

from __future__ import annotations

import sys
import time

import numpy as np

from paper_1107_4264_amd import synth

STREAM_SHAPE = (64, 2, 8, 128, 6)  # stations, pol, channels, chunk samples, chunks
BATCH_JOBS = [(20, 2, 6, 300), (70, 2, 5, 200), (128, 2, 4, 256), (150, 2, 3, 100), (9, 1, 7, 513)]
SINGLE = (128, 2, 16, 128)
DIST = ("gauss", 30.0, 127)


def inputs():
    ns, npol, F, chunk, nchunk = STREAM_SHAPE
    xs = synth.voltages_np(synth.SEED_BASE + 301, chunk * nchunk, F, ns * npol, DIST)
    xb = [synth.voltages_np(synth.SEED_BASE + 310 + k, t, f, s * p, DIST) for k, (s, p, f, t) in enumerate(BATCH_JOBS)]
    s, p, f, t = SINGLE
    x1 = synth.voltages_np(synth.SEED_BASE + 330, t, f, s * p, DIST)
    return xs, xb, x1


def run(delay_seed=None):
    """Returns {"stream": ..., "batch0": ..., ..., "single": ...} as numpy arrays."""
    import torch

    from paper_1107_4264_amd import xcorr as X

    rng = np.random.default_rng(delay_seed) if delay_seed is not None else None

    def pause():
        if rng is not None:
            time.sleep(float(rng.uniform(0.0, 0.003)))

    dev = torch.device("cuda:0")
    xs, xb, x1 = inputs()
    res = {}
    cur = torch.cuda.current_stream()
    side = torch.cuda.Stream()  # default priority

    # streaming: three pinned buffers, buffer p % 3 refilled once push p - 1 has returned
    ns, npol, F, chunk, nchunk = STREAM_SHAPE
    nin = ns * npol
    bufs = [torch.empty((chunk, F, nin, 2), dtype=torch.int8).pin_memory() for _ in range(3)]
    src = [torch.from_numpy(np.ascontiguousarray(xs[c * chunk:(c + 1) * chunk])) for c in range(nchunk)]
    st = X.Stream(ns, npol, F, chunk, "ci8", "i8")
    out = st.empty_out(dev)
    X.xcorr_stream_begin(st.s, out.data_ptr(), cur.cuda_stream)
    bufs[0].copy_(src[0])
    bufs[1].copy_(src[1])
    for p in range(nchunk):
        if p >= 2:
            pause()
            bufs[p % 3].copy_(src[p])
        pause()
        X.xcorr_stream_push(st.s, bufs[p % 3].data_ptr(), cur.cuda_stream)
    X.xcorr_stream_end(st.s, cur.cuda_stream)
    torch.cuda.synchronize()
    res["stream"] = out.cpu().numpy()
    st.close()

    # batch, launched three times with eager work on a second stream in between
    b = X.Batch(BATCH_JOBS, "ci8", "i8")
    xbt = [torch.from_numpy(x).to(dev) for x in xb]
    outs = b.empty_outs(dev)
    for rep in range(3):
        with torch.cuda.stream(side):
            junk = torch.randn(1 << 20, device=dev)
            junk.mul_(3.0).add_(1.0)
        pause()
        b.run(xbt, outs)
        pause()
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        res[f"batch{k}"] = o.cpu().numpy()
    b.close()

    # one job on the fp16 path, its input copied from pageable memory right before the run
    s, p, f, t = SINGLE
    c = X.Correlator(s, p, f, t, "ci8", "f16")
    xt = torch.empty(x1.shape, dtype=torch.int8, device=dev)
    xt.copy_(torch.from_numpy(x1), non_blocking=True)
    pause()
    res["single"] = c.run(xt).cpu().numpy()
    c.close()
    return res


if __name__ == "__main__":
    r = run(int(sys.argv[2]) if len(sys.argv) > 2 else None)
    np.savez(sys.argv[1], **r)
    print("race workload done", flush=True)
