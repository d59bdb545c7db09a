"""Benchmark of the MI355X X-engine on one GPU.

Workload: 128 stations x 2 polarisations (256 inputs), 1024 channels, 1000 samples per
integration, complex 8-bit samples drawn from a Gaussian of sigma 3, rounded and clipped
to [-127, 127] (seeded, synthetic; generated on the device).  A step is one full
X-engine pass (xcorr_run) over that input, resident in HBM.  Three arithmetic paths are
timed on the same input: the paper's FP32 complex MAC, FP16 MFMA with FP32 accumulation
(the headline value) and int8 MFMA with int32 accumulation.

Prints one JSON line.  Metric: X-engine TFLOPS = 8 flops per useful complex MAC (Eq. 5,
lower triangle including autocorrelations) / time.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

METRIC = "X-engine TFLOPS (8/CMAC) & % of peak: FP32 CMAC vs int8/FP16 MFMA, N=256 inputs"
# The headline workload and the compute-bound 4-bit one.  A step is one xcorr_run over the
# whole input, resident in HBM.
WORKLOADS = {
    "n256-ci8": {
        "name": "256 inputs (128 stations x 2 pol), 1024 channels, 1000 samples, ci8 gaussian sigma=3 clipped to +-127",
        "nstation": 128, "npol": 2, "nchan": 1024, "ntime": 1000, "in": "ci8",
        "dist": ("gauss", 3.0, 127), "seed_index": 1, "paths": "f32,f16,i8,f32m", "head": "f16",
        # the same arithmetic on other kernel shapes: 128-tiles staged in LDS against 128-tiles
        # whose waves load their operands through the caches (no LDS)
        "ablation": "f16:128,f16:128:cache,i8:128,i8:128:cache,f32m:128:cache",
    },
    "n1024-ci4": {
        "name": "1024 inputs (512 stations x 2 pol), 256 channels, 4096 samples, ci4 uniform [-8, 7]",
        "nstation": 512, "npol": 2, "nchan": 256, "ntime": 4096, "in": "ci4",
        "dist": ("uniform", -8, 7), "seed_index": 2, "paths": "i8,f8,f6", "head": "i8",
    },
}
PEAK_TFLOPS = {"f16": 2500.0, "i8": 5000.0, "f8": 5000.0, "f32": 157.3, "f32m": 157.3, "f6": 10100.0}


def parse_spec(spec):
    """Path spec acc[:tile][:cache][:vN]: arithmetic path, kernel tile (0: automatic), staging
    through the caches instead of LDS, compile-time kernel variant."""
    parts = spec.split(":")
    acc, tile, staging, variant = parts[0], 0, 0, 0
    for q in parts[1:]:
        if q == "cache":
            staging = 1
        elif q.startswith("v"):
            variant = int(q[1:])
        else:
            tile = int(q)
    return acc, tile, staging, variant
HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--ramp-seconds", type=float, default=0.3,
                    help="untimed run time per path before the warmup steps, so that clocks have settled")
    ap.add_argument("--workload", default="n256-ci8", choices=sorted(WORKLOADS) + ["batch64", "stream", "stream-full", "fengine"])
    ap.add_argument("--paths", default=None, help="comma-separated paths (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--only", default=None, help="time only this path (for profiling runs)")
    ap.add_argument("--tile", type=int, default=0,
                    help="kernel shape for the matrix-core paths: 0 automatic, 64/128 tiles, 256 whole channel")
    ap.add_argument("--no-small", action="store_true", help="skip the 64-input launch-latency figures")
    ap.add_argument("--no-ablation", action="store_true", help="skip the other kernel shapes of the workload")
    ap.add_argument("--no-autotune", action="store_true", help="run the planner's default shapes, not the autotuned ones")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one device copy of 1 GiB (reference for HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this X-engine build runs on one GPU; channels shard across GPUs "
                                   "with no exchange, but no multi-GPU run is provided"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1107_4264_amd import synth
    from paper_1107_4264_amd import xcorr as X

    dev = torch.device("cuda:0")
    if args.workload == "batch64":
        return bench_batch(args, dev)
    if args.workload in ("stream", "stream-full"):
        return bench_stream(args, dev, STREAM if args.workload == "stream" else STREAM_FULL)
    if args.workload == "fengine":
        print(json.dumps(bench_fengine(args, dev)), flush=True)
        return
    w = WORKLOADS[args.workload]
    ns, npol, F, T = w["nstation"], w["npol"], w["nchan"], w["ntime"]
    nin = ns * npol
    seed = synth.SEED_BASE + w["seed_index"]
    fmt = w["in"]
    in_enum = X.IN_CI8 if fmt == "ci8" else X.IN_CI4
    print(f"[bench] generating input {T}x{F}x{nin} {fmt} on device", file=sys.stderr, flush=True)
    x = synth.voltages_torch(seed, T, F, nin, w["dist"], dev)
    torch.cuda.synchronize()
    max_abs = int(x.abs().max().item())
    # the device generator reproduces the host definition (checked on one channel)
    chk = synth.voltages_np(seed, T, F, nin, w["dist"], chans=[F // 3])
    assert np.array_equal(x[:, F // 3: F // 3 + 1].cpu().numpy(), chk), "device generator mismatch"
    if fmt == "ci4":
        x = synth.pack_ci4_torch(x)
        torch.cuda.synchronize()

    paths = [p for p in (args.paths or w["paths"]).split(",") if p]
    if args.only:
        paths = [args.only]
    results = {}
    outs = {}
    stream = torch.cuda.current_stream()
    specs = list(paths)
    if not args.only and not args.no_ablation and w.get("ablation"):
        specs += w["ablation"].split(",")
    for p in specs:
        acc, tile, staging, variant = parse_spec(p)
        if tile == 0 and acc != "f32":
            tile = args.tile
        c = X.Correlator(ns, npol, F, T, fmt, acc, max_abs=max_abs, tile=tile or None, staging=staging or None,
                         variant=variant or None)
        out = c.empty_out(dev)
        tuned = None
        if p in paths and acc != "f32" and not args.tile and not args.no_autotune:
            # the paths of the workload run the shape the autotuner picks for them (every
            # tile x staging x variant the job allows, timed on the device), timed once the
            # clocks have ramped up under the default shape
            t_ramp = time.perf_counter()
            while time.perf_counter() - t_ramp < args.ramp_seconds:
                for _ in range(10):
                    c.run(x, out)
                torch.cuda.synchronize()
            c.autotune(x, out, reps=20)
            tuned = [{k: (round(v, 2) if isinstance(v, float) else v) for k, v in r.items()}
                     for r in X.xcorr_autotune_results(c.h)]
        plan = X.xcorr_plan(ns, npol, F, T, in_enum, X.ACC_NAMES[acc], max_abs, c.tile)
        # clocks ramp up under load: run the path untimed for a while, then the warmup steps
        t_ramp = time.perf_counter()
        while time.perf_counter() - t_ramp < args.ramp_seconds:
            for _ in range(10):
                c.run(x, out)
            torch.cuda.synchronize()
        for _ in range(args.warmup):
            c.run(x, out)
        torch.cuda.synchronize()
        steps = args.steps if p in paths else max(1, min(args.steps, 20))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            c.run(x, out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        useful = plan["useful_cmacs"]
        computed = plan["computed_cmacs"]
        tflops = 8.0 * useful / (ms * 1e-3) / 1e12
        alg_bytes = plan["in_bytes"] + plan["out_bytes"]
        results[p] = {
            "ms_per_step": ms,
            "tflops": tflops,
            "normalised_tflops": 8.0 * computed / (ms * 1e-3) / 1e12,
            "peak_tflops": PEAK_TFLOPS[acc],
            "frac_of_peak": tflops / PEAK_TFLOPS[acc],
            "algorithmic_gbps": alg_bytes / (ms * 1e-3) / 1e9,
            "out_type": ["ci32", "ci64", "c64", "c128"][plan["out_dtype"]],
            "windows": plan["nwindows"],
            "tile": plan["tile"],
            "staging": "caches" if c.staging else "lds",
            "variant": c.variant,
            "launches_per_step": launches_per_step(plan),
        }
        if tuned:
            results[p]["autotuned_from"] = tuned
        c.close()
        outs[p] = out
        print(f"[bench] {p}: {ms:.4f} ms/step, {tflops:.1f} TFLOPS", file=sys.stderr, flush=True)

    # the integer and the fp32 paths must agree exactly with each other on every value
    ref = None
    for p, o in outs.items():
        v = o.to(torch.float64)
        if ref is None:
            ref = v
        else:
            assert torch.equal(ref, v), f"path {p} disagrees with {list(outs)[0]}"

    if args.calibrate_copy:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    head = w["head"] if w["head"] in results else paths[0]
    hr = results[head]
    hacc = parse_spec(head)[0]
    plan = X.xcorr_plan(ns, npol, F, T, in_enum, X.ACC_NAMES[hacc], max_abs, hr["tile"])
    line = {
        "metric": METRIC,
        "value": round(hr["tflops"], 3),
        "unit": "TFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hr["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f16": "f16", "i8": "i8", "f32": "f32", "f8": "fp8", "f32m": "f32", "f6": "fp6"}[hacc],
        "data": "synthetic",
        "config": {"workload": w["name"], "nstation": ns, "npol": npol, "nchan": F, "ntime": T,
                   "in_dtype": fmt, "max_abs": max_abs, "tile": plan["tile"], "variant": hr["variant"],
                   "staging": hr["staging"],
                   "path": f"{head} mfma" if hacc != "f32" else "f32 cmac"},
        "roofline": {
            "bound": "mfma" if hacc != "f32" else "alu",
            "achieved": round(hr["tflops"], 3),
            "peak": PEAK_TFLOPS[hacc],
            "unit": "TFLOP/s",
            "frac": round(hr["frac_of_peak"], 4),
            "traffic": hbm_traffic(head, plan) if args.workload == "n256-ci8" and head == hacc else None,
        },
        "paths": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in r.items()}
                  for k, r in results.items()},
        "parity": "all timed paths agree exactly",
    }
    if "f32" in results and head != "f32":
        line["speedup_vs_f32_cmac"] = round(results["f32"]["ms_per_step"] / hr["ms_per_step"], 2)

    if not args.no_cpu_baseline and not args.only:
        line["cpu_baseline"], line["parity"] = cpu_baseline(args, w, outs[head], ns, npol, F, T, seed)
    if args.workload == "n256-ci8" and not args.only and not args.no_small:
        for k in list(outs):
            del outs[k]
        del x
        line["small_array"] = bench_small(args, dev)
        line["f_engine"] = bench_fengine(args, dev)
    print(json.dumps(line), flush=True)


FENGINE = {
    "name": "F-engine + corner turn: 256 inputs (128 stations x 2 pol), 1024-point transforms, 1000 frames "
            "(1,024,000 complex 8-bit samples per input, gaussian sigma=20), gain 0.5/sqrt(1024), requantised "
            "to 8-bit [frame][channel][input]",
    "nstation": 128, "npol": 2, "nchan": 1024, "nframes": 1000, "sigma": 20.0, "seed_index": 5,
}


def bench_fengine(args, dev):
    """The F-engine on the benchmark's X-engine input shape: time per pass, HBM bytes
    (input read once, requantised output written once) per second, and the FX chain (F-engine
    then the fp16 X-engine) per pass.  The CPU baseline leg runs the F-engine oracle on the
    first frames of every input and compares the requantised samples."""
    import numpy as np
    import torch

    from paper_1107_4264_amd import synth
    from paper_1107_4264_amd import xcorr as X

    w = FENGINE
    ns, npol, F, T = w["nstation"], w["npol"], w["nchan"], w["nframes"]
    nin = ns * npol
    seed = synth.SEED_BASE + w["seed_index"]
    dist = ("gauss", w["sigma"], 127)
    gain = 0.5 / F ** 0.5
    v = synth.voltages_torch(seed, T * F, 1, nin, dist, dev)          # [nsamp][1][nin][2]
    x = v[:, 0].permute(1, 0, 2).contiguous()                           # [nin][nsamp][2]
    del v
    e = X.FEngine(ns, npol, F, T, gain)
    out = e.empty_out(dev)
    c = X.Correlator(ns, npol, F, T, "ci8", "i8")
    vis = c.empty_out(dev)
    stream = torch.cuda.current_stream()
    steps = max(1, min(args.steps, 50))

    def timed(fn):
        for _ in range(max(args.warmup, 3)):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    ms_f = timed(lambda: e.run(x, out))
    ms_fx = timed(lambda: (e.run(x, out), c.run(out, vis)))
    nbytes = X.xcorr_fengine_in_bytes(e.e) + X.xcorr_fengine_out_bytes(e.e, 0)
    flops = 5.0 * F * np.log2(F) * nin * T
    res = {
        "workload": w["name"],
        "ms_per_pass": round(ms_f, 5),
        "hbm_gbps": round(nbytes / (ms_f * 1e-3) / 1e9, 1),
        "roofline": {"bound": "hbm", "achieved": round(nbytes / (ms_f * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(nbytes / (ms_f * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)},
        "fft_tflops": round(flops / (ms_f * 1e-3) / 1e12, 3),
        # the transform's 5 F log2 F flops against the fp32 vector peak: the kernel issues
        # several vector instructions per flop (conversions, requantisation, LDS addressing)
        "fft_frac_of_fp32_vector_peak": round(flops / (ms_f * 1e-3) / 1e12 / PEAK_TFLOPS["f32"], 4),
        "fx_chain_ms_per_pass": round(ms_fx, 5),
        "xengine_path": "i8 mfma (one int32 window, ci32 output)",
    }
    print(f"[bench] F-engine: {ms_f:.4f} ms per pass, {res['hbm_gbps']} GB/s; F + X: {ms_fx:.4f} ms",
          file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        from oracle import fengine as FE

        nf = 4  # first frames of every input (the generator's leading index is the sample)
        hv = synth.voltages_np(seed, nf * F, 1, nin, dist)
        hx = np.ascontiguousarray(np.transpose(hv[:, 0], (1, 0, 2)))
        t0 = time.perf_counter()
        spec = FE.channelise(hx, F, gain)
        want = FE.requantise(spec)
        dt = time.perf_counter() - t0
        got = out[:nf].cpu().numpy()
        diff = np.abs(got.astype(np.int16) - want)
        res["cpu_baseline"] = {"value": round(5.0 * F * np.log2(F) * nin * nf / dt / 1e12, 6), "unit": "TFLOPS",
                               "cores": 1, "kind": "oracle",
                               "sample": f"first {nf} frames of all {nin} inputs, {dt:.3f} s"}
        res["parity"] = (f"requantised samples of the sampled frames: {int((diff != 0).sum())} of {diff.size} "
                         f"components differ from the oracle, by at most {int(diff.max())} (fp32 against fp64 "
                         f"rounding at the half-integer boundaries)")
    e.close()
    c.close()
    return res


def launches_per_step(plan):
    """Kernel launches of one xcorr_run: the super-tiles run triangles and rectangles as two
    launches, the other kernels one; several windows add the zero fill of the wide output."""
    n = 2 if plan["tile"] == 512 else 1
    return n + (1 if plan["nwindows"] > 1 else 0)


SMALL = {
    "name": "64 inputs (32 stations x 2 pol), 16 channels, 256 samples, ci8 uniform [-8, 7]",
    "nstation": 32, "npol": 2, "nchan": 16, "ntime": 256, "dist": ("uniform", -8, 7), "seed_index": 0,
    "paths": ("f32", "i8", "f16"), "graph_runs": 100,
}


def bench_small(args, dev):
    """The small-array workload, where launch latency bounds the X-engine: per path the time
    of one launch in a stream of back-to-back launches, and the time per run when 100 runs
    are replayed from one captured HIP graph; algorithmic GB/s and TFLOPS from each.  The
    CPU baseline leg times the oracle on all channels and compares every path's output of
    both launch modes with it."""
    import numpy as np
    import torch

    from paper_1107_4264_amd import synth
    from paper_1107_4264_amd import xcorr as X

    w = SMALL
    ns, npol, F, T = w["nstation"], w["npol"], w["nchan"], w["ntime"]
    nin = ns * npol
    seed = synth.SEED_BASE + w["seed_index"]
    xh = synth.voltages_np(seed, T, F, nin, w["dist"])
    x = torch.from_numpy(xh).to(dev)
    res = {"workload": w["name"]}
    stream = torch.cuda.current_stream()
    steps = max(args.steps, 100)
    got = {}
    for p in w["paths"]:
        c = X.Correlator(ns, npol, F, T, "ci8", p, max_abs=8)
        plan = X.xcorr_plan(ns, npol, F, T, X.IN_CI8, X.ACC_NAMES[p], 8, 0)
        out = c.empty_out(dev)
        for _ in range(args.warmup + 10):
            c.run(x, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            c.run(x, out)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) / steps * 1e3
        got[p + " stream"] = out.cpu().numpy()
        # the same runs replayed from one captured graph
        g = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream()
        cs.wait_stream(stream)
        with torch.cuda.stream(cs):
            c.run(x, out)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=cs):
            for _ in range(w["graph_runs"]):
                c.run(x, out)
        torch.cuda.synchronize()
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        got[p + " graph"] = out.cpu().numpy()
        reps = 5
        e0.record(stream)
        for _ in range(reps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        us_graph = e0.elapsed_time(e1) / (reps * w["graph_runs"]) * 1e3
        alg = plan["in_bytes"] + plan["out_bytes"]
        useful = plan["useful_cmacs"]
        res[p] = {
            "us_per_launch": round(us, 3),
            "us_per_run_graph": round(us_graph, 3),
            "algorithmic_gbps": round(alg / (us * 1e-6) / 1e9, 2),
            "algorithmic_gbps_graph": round(alg / (us_graph * 1e-6) / 1e9, 2),
            "tflops": round(8.0 * useful / (us * 1e-6) / 1e12, 4),
            "tflops_graph": round(8.0 * useful / (us_graph * 1e-6) / 1e12, 4),
            "tile": plan["tile"],
        }
        print(f"[bench] small array {p}: {us:.2f} us per launch, {us_graph:.2f} us per run in a graph",
              file=sys.stderr, flush=True)
        del g
        c.close()
    res["algorithmic_bytes"] = alg
    res["useful_flops"] = 8 * useful
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        t0 = time.perf_counter()
        want = oracle.xcorr(xh, ns, npol)
        dt = time.perf_counter() - t0
        bad = [k for k, v in got.items() if not np.array_equal(np.rint(v).astype(np.int64), want)]
        res["cpu_baseline"] = {"value": round(8.0 * useful / dt / 1e12, 6), "unit": "TFLOPS",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "sample": f"all {F} channels, {dt * 1e3:.2f} ms wall"}
        res["parity"] = ("every path, launched alone and replayed from the graph, bit-exact against the oracle"
                         if not bad else "MISMATCH against the oracle: " + ", ".join(bad))
    return res


BATCH = {
    "name": "64 uneven jobs: inputs 2*U{24..288} (dual pol), 32..512 channels, 128..8192 samples, "
            "ci8 gaussian sigma=8 clipped to +-127",
    "seed_index": 3, "dist": ("gauss", 8.0, 127), "path": "i8",
}


def bench_batch(args, dev):
    """All jobs in one persistent launch against one launch per job (each with its own
    automatic kernel shape); value = useful TFLOPS of the persistent launch."""
    import numpy as np
    import torch

    from paper_1107_4264_amd import synth
    from paper_1107_4264_amd import xcorr as X

    seed = synth.SEED_BASE + BATCH["seed_index"]
    jobs = synth.draw_jobs(seed)
    acc = BATCH["path"]
    print(f"[bench] generating {len(jobs)} job inputs on device", file=sys.stderr, flush=True)
    xs = [synth.voltages_torch(seed + 16 * (k + 1), j["ntime"], j["nchan"], j["nstation"] * j["npol"],
                               BATCH["dist"], dev) for k, j in enumerate(jobs)]
    torch.cuda.synchronize()
    max_abs = max(int(x.abs().max().item()) for x in xs)
    useful = sum((j["nstation"] * j["npol"]) * (j["nstation"] * j["npol"] + 1) // 2 * j["nchan"] * j["ntime"]
                 for j in jobs)
    in_bytes = sum(x.numel() for x in xs)
    stream = torch.cuda.current_stream()

    def timed(fn):
        t_ramp = time.perf_counter()
        while time.perf_counter() - t_ramp < args.ramp_seconds:
            fn()
            torch.cuda.synchronize()
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    b = X.Batch(jobs, "ci8", acc, max_abs=max_abs)
    outs_b = b.empty_outs(dev)
    ms_batch = timed(lambda: b.run(xs, outs_b))
    print(f"[bench] batch: {ms_batch:.3f} ms/step, {8.0 * useful / (ms_batch * 1e-3) / 1e12:.1f} TFLOPS",
          file=sys.stderr, flush=True)
    cs = [X.Correlator(j["nstation"], j["npol"], j["nchan"], j["ntime"], "ci8", acc, max_abs=max_abs) for j in jobs]
    outs_j = [c.empty_out(dev) for c in cs]

    def per_job():
        for c, x, o in zip(cs, xs, outs_j):
            c.run(x, o)

    ms_jobs = timed(per_job)
    print(f"[bench] per-job launches: {ms_jobs:.3f} ms/step", file=sys.stderr, flush=True)
    same = all(torch.equal(a, bb) for a, bb in zip(outs_b, outs_j))
    tiles = sorted({c.tile for c in cs})
    tflops = 8.0 * useful / (ms_batch * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": round(tflops, 3), "unit": "TFLOPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_batch, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i8", "data": "synthetic",
        "config": {"workload": BATCH["name"], "jobs": len(jobs), "useful_cmacs": useful, "in_bytes": in_bytes,
                   "max_abs": max_abs, "path": "i8 mfma, one persistent launch"},
        "roofline": {"bound": "mfma", "achieved": round(tflops, 3), "peak": PEAK_TFLOPS["i8"], "unit": "TFLOP/s",
                     "frac": round(tflops / PEAK_TFLOPS["i8"], 4), "traffic": None},
        "per_job_launches": {"ms_per_step": round(ms_jobs, 5), "tflops": round(8.0 * useful / (ms_jobs * 1e-3) / 1e12, 3),
                             "tiles": tiles},
        "batch_speedup_vs_per_job": round(ms_jobs / ms_batch, 3),
        "parity": "persistent and per-job launches agree exactly" if same else "MISMATCH between launch modes",
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"], ok = batch_cpu_baseline(args, jobs, seed, outs_b)
        line["parity"] += "; sampled channels bit-exact against the oracle" if ok else "; MISMATCH against the oracle"
    print(json.dumps(line), flush=True)


STREAM = {
    "name": "streaming integration: 1024 inputs (512 stations x 2 pol), 512 channels, 16 chunks of 4096 samples "
            "from a pool of 2 pinned host chunks, ci8 gaussian sigma=20 clipped to +-127",
    "nstation": 512, "npol": 2, "nchan": 512, "chunk": 4096, "nchunk": 16, "pool": 2,
    "dist": ("gauss", 20.0, 127), "seed_index": 4, "path": "i8",
}

# The same integration at its full size: 4096 channels, 34.4 GB per chunk (two pinned host
# chunks of 2^35 bytes, 549.8 GB copied per integration).
STREAM_FULL = dict(STREAM, nchan=4096,
                   name="streaming integration: 1024 inputs (512 stations x 2 pol), 4096 channels, 16 chunks of 4096 "
                        "samples (65536 samples) from a pool of 2 pinned host chunks, ci8 gaussian sigma=20 clipped "
                        "to +-127")


def bench_stream(args, dev, w):
    """End-to-end chunked integration from pinned host memory (copies overlapped with the
    X-engine); a step is the whole integration, wall time includes the host-to-device copies."""
    import numpy as np
    import torch

    from paper_1107_4264_amd import synth
    from paper_1107_4264_amd import xcorr as X

    ns, npol, F, C = w["nstation"], w["npol"], w["nchan"], w["chunk"]
    nin = ns * npol
    seed = synth.SEED_BASE + w["seed_index"]
    pool = []
    for k in range(w["pool"]):
        print(f"[bench] generating pinned chunk {k} ({C}x{F}x{nin} ci8)", file=sys.stderr, flush=True)
        d = synth.voltages_torch(seed, C, F, nin, w["dist"], dev, t0=k * C)
        h = torch.empty(d.shape, dtype=torch.int8, pin_memory=True)
        h.copy_(d)
        pool.append(h)
        del d
    torch.cuda.synchronize()
    st = X.Stream(ns, npol, F, C, "ci8", w["path"])
    out = st.empty_out(dev)
    chunk_bytes = pool[0].numel()
    useful = nin * (nin + 1) // 2 * F * C * w["nchunk"]

    def integrate():
        st.begin(out)
        for c in range(w["nchunk"]):
            st.push(pool[c % w["pool"]])
        st.end()

    steps = max(1, min(args.steps, 3))
    integrate()
    torch.cuda.synchronize()
    print("[bench] warm-up integration done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for k in range(steps):
        integrate()
        print(f"[bench] integration {k} issued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    # the X-engine alone on one resident chunk, for the overlap figure
    c1 = X.Correlator(ns, npol, F, C, "ci8", w["path"])
    xd = pool[0].to(dev)
    o1 = c1.empty_out(dev)
    for _ in range(3):
        c1.run(xd, o1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        c1.run(xd, o1)
    e1.record()
    torch.cuda.synchronize()
    kern_ms = e0.elapsed_time(e1) / 5
    h2d = chunk_bytes * w["nchunk"] / wall / 1e9
    tflops = 8.0 * useful / wall / 1e12
    print(f"[bench] stream: {wall * 1e3:.1f} ms per integration, {h2d:.1f} GB/s host to device, "
          f"X-engine {kern_ms:.2f} ms per chunk", file=sys.stderr, flush=True)
    line = {
        "metric": METRIC, "value": round(tflops, 3), "unit": "TFLOPS", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": round(wall * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "i8", "data": "synthetic",
        "config": {"workload": w["name"], "chunk_bytes": chunk_bytes, "path": "i8 mfma streaming, int64 totals"},
        "roofline": {"bound": "host link", "achieved": round(h2d, 2), "peak": None, "unit": "GB/s", "frac": None,
                     "traffic": None},
        "xengine_ms_per_chunk": round(kern_ms, 4),
        "copy_ms_per_chunk": round(wall * 1e3 / w["nchunk"], 4),
    }
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        chans = [0, F // 2, F - 1]
        got = out[chans].cpu().numpy()
        want = np.zeros_like(got, dtype=np.int64)
        t0 = time.perf_counter()
        for k in range(w["pool"]):
            xk = synth.voltages_np(seed, C, F, nin, w["dist"], t0=k * C, chans=chans)
            want += oracle.xcorr(xk, ns, npol, chans=np.arange(len(chans))) * (w["nchunk"] // w["pool"])
        dt = time.perf_counter() - t0
        ok = np.array_equal(got.astype(np.int64), want)
        line["cpu_baseline"] = {"value": round(8.0 * nin * (nin + 1) // 2 * len(chans) * C * w["pool"] / dt / 1e12, 6),
                                "unit": "TFLOPS", "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"channels {chans} of the {w['pool']} pool chunks, {dt:.2f} s"}
        line["parity"] = ("totals equal the sum of the chunks' oracle visibilities (linearity) on sampled channels"
                          if ok else "MISMATCH against the oracle")
    print(json.dumps(line), flush=True)


def batch_cpu_baseline(args, jobs, seed, outs):
    """The oracle on one channel of jobs taken in a seeded random order until the CPU time
    budget is spent."""
    import numpy as np

    import oracle
    from paper_1107_4264_amd import synth

    oracle.build()
    rng = np.random.default_rng(1)
    order = [int(k) for k in rng.permutation(len(jobs))]
    spent, useful, ok, done = 0.0, 0, True, []
    for k in order:
        if spent > args.cpu_seconds and done:
            break
        j = jobs[k]
        nin = j["nstation"] * j["npol"]
        f = int(rng.integers(j["nchan"]))
        x = synth.voltages_np(seed + 16 * (k + 1), j["ntime"], j["nchan"], nin, BATCH["dist"], chans=[f])
        t0 = time.perf_counter()
        want = oracle.xcorr(x, j["nstation"], j["npol"], chans=[0])
        spent += time.perf_counter() - t0
        useful += nin * (nin + 1) // 2 * j["ntime"]
        ok = ok and np.array_equal(outs[k][f:f + 1].cpu().numpy().astype(np.int64), want)
        done.append(f"job {int(k)} channel {f}")
    base = {"value": round(8.0 * useful / spent / 1e12, 6), "unit": "TFLOPS", "cores": 1, "kind": "oracle",
            "sample": f"one channel of {len(done)} jobs ({', '.join(done)}), {spent:.2f} s"}
    return base, ok


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "xeng_chan_256in_1024ch_1000t_hbm_traffic.json")


def hbm_traffic(path, plan):
    """HBM bytes per launch of the path's kernel, from the counter runs recorded in
    TRAFFIC_FILE (FETCH_SIZE and WRITE_SIZE, scaled by their calibration against kernels of
    known traffic), if they were taken on the current kernel source; otherwise None."""
    import hashlib

    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    here = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    entry = rec["paths"].get(path)
    if h.hexdigest() != rec["sources_sha256"] or entry is None or plan["tile"] != rec["tile"]:
        return None
    return int(entry["fetch_kib"] * 1024 * rec["fetch_factor"] + entry["write_kib"] * 1024 * rec["write_factor"])


def cpu_baseline(args, w, out_head, ns, npol, F, T, seed):
    """The oracle on a bounded sample of channels of the same workload, on the host cores;
    the sampled channels are also compared with the GPU output."""
    import numpy as np

    import oracle
    from paper_1107_4264_amd import synth

    oracle.build()
    nin = ns * npol
    ci4 = w["in"] == "ci4"

    def host_input(chans):
        v = synth.voltages_np(seed, T, F, nin, w["dist"], chans=chans)
        return synth.pack_ci4(v) if ci4 else v

    ofmt = oracle.CI4 if ci4 else oracle.CI8
    cores = oracle.num_threads()
    # size the sample: time one channel first
    rng = np.random.default_rng(0)
    first = [int(rng.integers(F))]
    xs = host_input(first)
    t0 = time.perf_counter()
    oracle.xcorr(xs, ns, npol, fmt=ofmt, chans=[0])
    one = time.perf_counter() - t0
    nsel = min(F, max(1, cores * max(1, int(args.cpu_seconds / max(one, 1e-6)))))
    chans = np.sort(rng.choice(F, size=nsel, replace=False))
    xs = host_input(chans)
    t0 = time.perf_counter()
    want = oracle.xcorr(xs, ns, npol, fmt=ofmt, chans=np.arange(nsel))
    dt = time.perf_counter() - t0
    useful = nin * (nin + 1) // 2 * nsel * T
    got = out_head[chans.tolist()].cpu().numpy()
    exact = np.array_equal(np.rint(got).astype(np.int64), want) and np.array_equal(np.rint(got), got)
    base = {
        "value": round(8.0 * useful / dt / 1e12, 6),
        "unit": "TFLOPS",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{nsel} of {F} channels (all {T} samples, all {nin*(nin+1)//2} input pairs), {dt:.2f} s wall",
    }
    parity = (f"all timed paths agree exactly; headline path bit-exact against the oracle on "
              f"{nsel} sampled channels" if exact else "MISMATCH against the oracle on sampled channels")
    if not exact:
        print("[bench] PARITY FAILURE on sampled channels", file=sys.stderr, flush=True)
    return base, parity


if __name__ == "__main__":
    main()
