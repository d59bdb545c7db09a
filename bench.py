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
        "dist": ("gauss", 3.0, 127), "seed_index": 1, "paths": "f32,f16,i8", "head": "f16",
    },
    "n1024-ci4": {
        "name": "1024 inputs (512 stations x 2 pol), 256 channels, 4096 samples, ci4 uniform [-8, 7]",
        "nstation": 512, "npol": 2, "nchan": 256, "ntime": 4096, "in": "ci4",
        "dist": ("uniform", -8, 7), "seed_index": 2, "paths": "i8,f8", "head": "i8",
    },
}
PEAK_TFLOPS = {"f16": 2500.0, "i8": 5000.0, "f8": 5000.0, "f32": 157.3}
HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--ramp-seconds", type=float, default=0.3,
                    help="untimed run time per path before the warmup steps, so that clocks have settled")
    ap.add_argument("--workload", default="n256-ci8", choices=sorted(WORKLOADS))
    ap.add_argument("--paths", default=None, help="comma-separated paths (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--only", default=None, help="time only this path (for profiling runs)")
    ap.add_argument("--tile", type=int, default=0,
                    help="kernel shape for the matrix-core paths: 0 automatic, 64/128 tiles, 256 whole channel")
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
    for p in paths:
        tile = args.tile if p != "f32" else 0
        c = X.Correlator(ns, npol, F, T, fmt, p, max_abs=max_abs, tile=tile)
        plan = X.xcorr_plan(ns, npol, F, T, in_enum, X.ACC_NAMES[p], max_abs, tile)
        out = c.empty_out(dev)
        # clocks ramp up under load: run the path untimed for a while, then the warmup steps
        t_ramp = time.perf_counter()
        while time.perf_counter() - t_ramp < args.ramp_seconds:
            for _ in range(10):
                c.run(x, out)
            torch.cuda.synchronize()
        for _ in range(args.warmup):
            c.run(x, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            c.run(x, out)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        useful = plan["useful_cmacs"]
        computed = plan["computed_cmacs"]
        tflops = 8.0 * useful / (ms * 1e-3) / 1e12
        alg_bytes = plan["in_bytes"] + plan["out_bytes"]
        results[p] = {
            "ms_per_step": ms,
            "tflops": tflops,
            "normalised_tflops": 8.0 * computed / (ms * 1e-3) / 1e12,
            "peak_tflops": PEAK_TFLOPS[p],
            "frac_of_peak": tflops / PEAK_TFLOPS[p],
            "algorithmic_gbps": alg_bytes / (ms * 1e-3) / 1e9,
            "out_type": ["ci32", "ci64", "c64", "c128"][plan["out_dtype"]],
            "windows": plan["nwindows"],
            "tile": plan["tile"],
            "launches_per_step": 1 if plan["nwindows"] == 1 else 2,
        }
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
    plan = X.xcorr_plan(ns, npol, F, T, in_enum, X.ACC_NAMES[head], max_abs, args.tile if head != "f32" else 0)
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
        "dtype": {"f16": "f16", "i8": "i8", "f32": "f32", "f8": "fp8"}[head],
        "data": "synthetic",
        "config": {"workload": w["name"], "nstation": ns, "npol": npol, "nchan": F, "ntime": T,
                   "in_dtype": fmt, "max_abs": max_abs, "tile": plan["tile"],
                   "path": f"{head} mfma" if head != "f32" else "f32 cmac"},
        "roofline": {
            "bound": "mfma" if head != "f32" else "alu",
            "achieved": round(hr["tflops"], 3),
            "peak": PEAK_TFLOPS[head],
            "unit": "TFLOP/s",
            "frac": round(hr["frac_of_peak"], 4),
            "traffic": hbm_traffic(head, plan) if args.workload == "n256-ci8" else None,
        },
        "paths": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in r.items()}
                  for k, r in results.items()},
        "parity": "all timed paths agree exactly",
    }
    if "f32" in results and head != "f32":
        line["speedup_vs_f32_cmac"] = round(results["f32"]["ms_per_step"] / hr["ms_per_step"], 2)

    if not args.no_cpu_baseline and not args.only:
        line["cpu_baseline"], line["parity"] = cpu_baseline(args, w, outs[head], ns, npol, F, T, seed)
    print(json.dumps(line), flush=True)


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
