#!/usr/bin/env python3
"""Benchmark of the stencil sweep on one MI355X.

Workload (one "step" = one whole sweep of the workload through the library):
  Box-2D3R (49 points) and Star-2D3R (13 points), 8192 x 8192 grid, float64
  and float32, values uniform on [0, 1), random weights normalised to sum 1,
  zero Dirichlet halo, 100 time steps per sweep, fusion depth T in {1, 2, 4},
  VALU and MFMA paths.  The headline line is Box-2D3R float64 at the fastest
  (path, T); every variant is listed under "variants".

GStencil/s = grid points x time steps / seconds / 1e9, with the grids resident
in HBM before the timed region.  Kernel time comes from HIP events recorded on
the stream the library launches on.

The roofline object describes the headline variant's kernel: achieved =
algorithmic bytes per launch (2 D per point: one read, one write) or
algorithmic flops per launch (2 K T per point), divided by the average launch
duration; the bound is the one the performance model assigns (HBM when the
VALU intensity T K / D is below the ridge, otherwise the vector-ALU peak).

cpu_baseline: the FP64 oracle (plain C, OpenMP) timed on the host on a bounded
sample of the same workload (a few time steps of the full grid).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12           # bytes/s
PEAK_VALU_F64 = 78.6e12     # flop/s, FP64 vector FMA (256 CU x 2.4 GHz x 128)
PEAK_VALU_F32 = 78.6e12     # flop/s, scalar FP32 FMA (packed forms not issued)
PEAK_MFMA = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2516.6e12, "f16": 2516.6e12}
DBYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2, "bf16x3": 4}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed sweeps per variant")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--time-steps", type=int, default=100, help="stencil steps per sweep")
    ap.add_argument("--n", type=int, default=8192, help="grid side")
    ap.add_argument("--only", default="", help="comma list of variant names to run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--json-out", default="")
    return ap.parse_args()


def variants(n, nsteps):
    out = []
    for shape, K in (("box", 49), ("star", 13)):
        for dt in ("f64", "f32"):
            for T in (1, 2, 4):
                for path in ("valu", "mfma"):
                    name = f"{shape}-2d3r-{dt}-T{T}-{path}"
                    out.append(dict(name=name, shape=shape, K=K, d=2, r=3, dtype=dt, T=T,
                                    path=path, dims=(n, n), steps=nsteps))
    return out


def time_variant(stl, v, x, w, steps, warmup):
    import torch

    try:
        p = stl.Plan(v["shape"], v["d"], v["r"], w, v["dims"], T=v["T"], dtype=v["dtype"],
                     path=v["path"])
    except stl.StencilError as e:
        return dict(error=str(e))
    info = p.info()
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        p.run(x, y, v["steps"], stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        p.run(x, y, v["steps"], stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    npts = v["dims"][0] * v["dims"][1]
    gst = npts * v["steps"] / (ms * 1e-3) / 1e9
    passes = (v["steps"] + v["T"] - 1) // v["T"]
    launch_ms = ms / passes
    D = DBYTES[v["dtype"]]
    bytes_per_launch = 2.0 * D * npts
    flops_per_launch = 2.0 * v["K"] * v["T"] * npts
    # model bound of the VALU path: HBM below the ridge, vector ALU above it
    peak_alu = PEAK_VALU_F64 if v["dtype"] == "f64" else PEAK_VALU_F32
    I = v["T"] * v["K"] / D
    if I < peak_alu / PEAK_HBM:
        roof = dict(bound="hbm", achieved=bytes_per_launch / (launch_ms * 1e-3) / 1e9,
                    peak=PEAK_HBM / 1e9, unit="GB/s")
    else:
        roof = dict(bound="alu", achieved=flops_per_launch / (launch_ms * 1e-3) / 1e12,
                    peak=peak_alu / 1e12, unit="TFLOP/s")
    if info["path"] == 2:  # MFMA path: useful flops against the matrix peak
        I_exec = I * info["gamma"] * info["alpha"] / info["S"]
        pk = PEAK_MFMA[v["dtype"]]
        if I_exec >= pk / PEAK_HBM:
            roof = dict(bound="mfma", achieved=flops_per_launch * info["gamma"] * info["alpha"] /
                        info["S"] / (launch_ms * 1e-3) / 1e12, peak=pk / 1e12, unit="TFLOP/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    p.close()
    return dict(ms_per_sweep=ms, gst=gst, launch_ms=launch_ms, passes=passes, roofline=roof,
                path=info["path_name"], predicted_gst=info["predicted_gst_valu"] if info["path"] == 1
                else info["predicted_gst_mfma"], predicted_winner=info["predicted_winner"],
                scenario=info["scenario"], S=info["S"], alpha=info["alpha"])


def cpu_baseline(n, budget_s):
    """Oracle on the full grid for as many time steps as fit the budget."""
    import numpy as np

    import stencil_inputs as si
    from oracle import core

    w = si.normalised_weights(49, seed=si.weight_seed(2, 0))
    u0 = si.uniform_grid((n, n), seed=si.data_seed(2, 0))
    threads = core.max_threads()
    t0 = time.perf_counter()
    core.run("box", 2, 3, w, u0, 1, "dirichlet", 0.0)
    t1 = time.perf_counter()
    one = t1 - t0
    k = max(1, min(20, int(budget_s / max(one, 1e-3)) - 1))
    t0 = time.perf_counter()
    core.run("box", 2, 3, w, u0, k, "dirichlet", 0.0)
    dt = time.perf_counter() - t0
    return dict(value=n * n * k / dt / 1e9, unit="GStencil/s", cores=threads, kind="oracle",
                sample=f"Box-2D3R f64 {n}x{n}, {k} time steps (of 100), zero Dirichlet halo")


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the stencil library has no multi-GPU path "
              "(a grid would shard as slabs along its slowest axis with r*T-deep halo "
              "exchange per pass); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2603_00477_amd as stl
    import stencil_inputs as si

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stl.lib()
    n = args.n
    vs = variants(n, args.time_steps)
    if args.only:
        keep = set(args.only.split(","))
        vs = [v for v in vs if v["name"] in keep]
    u0 = si.uniform_grid((n, n), seed=si.data_seed(2, 0))
    inputs = {}
    results = {}
    for v in vs:
        key = v["dtype"]
        if key not in inputs:
            inputs[key] = si.round_to(u0, key)[1].to("cuda")
        w = si.normalised_weights(v["K"], seed=si.weight_seed(2, 0 if v["shape"] == "box" else 1))
        r = time_variant(stl, v, inputs[key], w, args.steps, args.warmup)
        results[v["name"]] = r
        print(f"# {v['name']}: " + (f"{r['gst']:.1f} GSt/s, {r['roofline']['frac']:.3f} of "
              f"{r['roofline']['bound']}" if "gst" in r else r.get("error", "?")), file=sys.stderr,
              flush=True)
    ok = {k: r for k, r in results.items() if "gst" in r}
    box64 = {k: r for k, r in ok.items() if k.startswith("box-2d3r-f64")}
    head_name = max(box64 or ok, key=lambda k: (box64 or ok)[k]["gst"])
    head = ok[head_name]
    hv = next(v for v in vs if v["name"] == head_name)
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(n, args.cpu_seconds)
    line = {
        "metric": "GStencil/s (Box-2D3R 8192^2 f64, 100 steps, best path/T)",
        "value": head["gst"],
        "unit": "GStencil/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_sweep"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": hv["dtype"],
        "data": "synthetic",
        "config": {"workload": f"{hv['shape'].capitalize()}-2D3R {n}x{n} {hv['dtype']}, "
                               f"{args.time_steps} steps, Dirichlet h=0, T={hv['T']}, "
                               f"{head['path']} path",
                   "grid": [n, n], "time_steps": args.time_steps, "T": hv["T"],
                   "path": head["path"]},
        "roofline": dict(head["roofline"], traffic=None),
        "cpu_baseline": cpu,
        "variants": {k: {kk: r[kk] for kk in ("gst", "path", "predicted_gst", "predicted_winner",
                                               "scenario", "launch_ms")}
                     | {"frac": r["roofline"]["frac"], "bound": r["roofline"]["bound"]}
                     for k, r in ok.items()},
    }
    s = json.dumps(line)
    print(s, flush=True)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(s + "\n")


if __name__ == "__main__":
    main()
