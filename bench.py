#!/usr/bin/env python3
"""Benchmark of the stencil sweeps on one MI355X.

Headline (one "step" = one whole sweep of the workload through the library):
  Box-2D3R (49 points) and Star-2D3R (13 points), 8192 x 8192, float64 and
  float32, U[0,1) data, random weights normalised to sum 1, zero Dirichlet
  halo, 100 time steps per sweep, fusion depth T in {1, 2, 4}, VALU and MFMA
  paths.  The JSON line's value is Box-2D3R float64 at the fastest (path, T).

Further sections (extra keys of the same JSON line):
  model_check  the 3D workload (Star-3D2R, Box-3D1R, 512^3, periodic, 50
               steps, T in {1,2,3}) plus the 8192^2 variants: the model's
               predicted winner (VALU / tie / MFMA, tie band 0.87-1.15) next
               to the measured one.
  precision    Box-2D2R, 16384^2, periodic, 1000 steps, smooth
               sin(2 pi x) sin(2 pi y) + 1e-3 U[0,1) data: bf16 / f16 MFMA with
               float32 accumulation, compensated bf16x3, VALU comparators;
               relative max-norm error against the float64 GPU sweep every 100
               steps, and GStencil/s.
  serving      served stream (4096 jobs, Poisson arrivals, mixed shape/d/r/
               size/steps, float32, HBM budget): continuous-batching server vs
               one-plan-per-call FIFO on the same trace; p50/p99 latency and
               aggregate GStencil/s.
  paper_cases  the six cases of the paper's Table 3 at 10240^2 / 1024^3 on
               both paths, predicted vs measured winner.

GStencil/s = grid points x time steps / seconds / 1e9 (grids resident in HBM
before the timed region).  Kernel time comes from HIP events recorded on the
stream the library launches on.

roofline (headline kernel): achieved = algorithmic bytes per launch (2 D per
point: one read, one write) or algorithmic flops per launch (2 K T per point)
divided by the average launch duration; the bound is the one the model
assigns to the VALU path (HBM below the ridge T K / D < PP/BB, else the
vector-ALU peak: 78.6 TFLOP/s FP64, 157.3 TFLOP/s FP32).  traffic: HBM bytes per launch from the
rocprofv3 FETCH_SIZE / WRITE_SIZE summaries under profiles/, scaled by the
same counters on a copy of known size; null when the kernel sources changed
since those counters were taken.

cpu_baseline: the FP64 oracle (plain C, OpenMP) on the host, on a bounded
sample of the headline workload (a few time steps of the full grid).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12           # bytes/s
PEAK_VALU = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 157.3e12, "f16": 157.3e12}
# flop/s: 256 CU x 2.4 GHz x (64 FP64 | 128 FP32) FMA lanes per clock x 2
PEAK_MFMA = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2516.6e12, "f16": 2516.6e12,
             "bf16x3": 2516.6e12}
DBYTES = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2, "bf16x3": 4}
KERNEL_SOURCES = ["paper_2603_00477_amd/csrc/valu2d_impl.h", "paper_2603_00477_amd/csrc/valu_common.h"]


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed sweeps per variant")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--time-steps", type=int, default=100, help="stencil steps per sweep")
    ap.add_argument("--n", type=int, default=8192, help="grid side of the headline workload")
    ap.add_argument("--only", default="", help="comma list of headline variant names to run")
    ap.add_argument("--sections", default="c2,c3,c4,c5,cases,sparse,grid,seq")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-clocks", action="store_true",
                    help="skip the rocm-smi clock reading (runs under a profiler, which may not start "
                         "other programs)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--jobs", type=int, default=4096, help="served-stream jobs")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain device copy of the headline grid (counter calibration)")
    ap.add_argument("--json-out", default="")
    return ap.parse_args()


# ---------------------------------------------------------------- timing
def timed_runs(p, x, y, nsteps, reps, warmup):
    import torch

    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        p.run(x, y, nsteps, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        p.run(x, y, nsteps, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def roofline_for(v, info, launch_ms, npts):
    D = DBYTES[v["dtype"]]
    T = info["T"]
    K = info["K"]
    bytes_per_launch = 2.0 * D * npts
    flops_per_launch = 2.0 * K * T * npts
    if info["path"] == 2:  # MFMA: executed flops against the matrix peak when above its ridge
        I_exec = T * K / D * info["gamma"] * info["alpha"] / info["S"]
        pk = PEAK_MFMA[v["dtype"]]
        if I_exec >= pk / PEAK_HBM:
            ach = flops_per_launch * info["gamma"] * info["alpha"] / info["S"] / (launch_ms * 1e-3)
            return dict(bound="mfma", achieved=ach / 1e12, peak=pk / 1e12, unit="TFLOP/s",
                        frac=ach / pk)
    elif T * K / D >= PEAK_VALU[v["dtype"]] / PEAK_HBM:
        pk = PEAK_VALU[v["dtype"]]
        ach = flops_per_launch / (launch_ms * 1e-3)
        return dict(bound="alu", achieved=ach / 1e12, peak=pk / 1e12, unit="TFLOP/s", frac=ach / pk)
    ach = bytes_per_launch / (launch_ms * 1e-3)
    return dict(bound="hbm", achieved=ach / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s", frac=ach / PEAK_HBM)


def measure(stl, v, x, w, reps, warmup):
    import torch

    try:
        p = stl.Plan(v["shape"], v["d"], v["r"], w, v["dims"], T=v["T"], dtype=v["dtype"],
                     path=v["path"], boundary=v.get("boundary", "dirichlet"))
    except stl.StencilError as e:
        return dict(error=str(e))
    info = p.info()
    y = torch.empty_like(x)
    ms = timed_runs(p, x, y, v["steps"], reps, warmup)
    npts = math.prod(v["dims"])
    passes = -(-v["steps"] // v["T"])
    launch_ms = ms / passes
    out = dict(ms_per_sweep=ms, gst=npts * v["steps"] / (ms * 1e-3) / 1e9, launch_ms=launch_ms,
               path=info["path_name"], T=info["T"], S=info["S"], alpha=info["alpha"],
               scenario=info["scenario"], predicted_winner=info["predicted_winner"],
               predicted_gst=info["predicted_gst_valu"] if info["path"] == 1 else info["predicted_gst_mfma"],
               roofline=roofline_for(v, info, launch_ms, npts))
    p.close()
    del y
    return out


def verdict(ratio):
    return "mfma" if ratio > 1.15 else ("valu" if ratio < 0.87 else "tie")


# ---------------------------------------------------------------- 8192^2 2D workload
def headline_variants(n, nsteps):
    out = []
    for shape, K in (("box", 49), ("star", 13)):
        for dt in ("f64", "f32"):
            for T in (1, 2, 4):
                for path in ("valu", "mfma"):
                    out.append(dict(name=f"{shape}-2d3r-{dt}-T{T}-{path}", shape=shape, K=K, d=2, r=3,
                                    dtype=dt, T=T, path=path, dims=(n, n), steps=nsteps))
    return out


def section_c2(stl, args):
    import torch

    import stencil_inputs as si

    n = args.n
    vs = headline_variants(n, args.time_steps)
    if args.only:
        keep = set(args.only.split(","))
        vs = [v for v in vs if v["name"] in keep]
    u0 = si.uniform_grid((n, n), seed=si.data_seed(2, 0))
    inputs, results = {}, {}
    for v in vs:
        if v["dtype"] not in inputs:
            inputs[v["dtype"]] = si.round_to(u0, v["dtype"])[1].to("cuda")
        w = si.normalised_weights(v["K"], seed=si.weight_seed(2, 0 if v["shape"] == "box" else 1))
        r = measure(stl, v, inputs[v["dtype"]], w, args.steps, args.warmup)
        results[v["name"]] = r
        log(f"{v['name']}: " + (f"{r['gst']:.1f} GSt/s, {r['roofline']['frac']:.3f} of "
                                 f"{r['roofline']['bound']}" if "gst" in r else r.get("error", "?")))
    if args.calib_copy:
        x = inputs.get("f64", next(iter(inputs.values())))
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"calibration copy: {x.numel() * x.element_size()} bytes read and written per copy")
    del inputs
    torch.cuda.empty_cache()
    return results


# ---------------------------------------------------------------- 512^3 3D workload
def section_c3(stl, args):
    import torch

    import stencil_inputs as si

    n = 512
    res = {}
    u0 = si.uniform_grid((n, n, n), seed=si.data_seed(3, 0))
    for dt in ("f64", "f32"):
        x = si.round_to(u0, dt)[1].to("cuda")
        for vi, (shape, r, K) in enumerate((("star", 2, 13), ("box", 1, 27))):
            w = si.normalised_weights(K, seed=si.weight_seed(3, vi))
            for T in (1, 2, 3):
                row = {}
                for path in ("valu", "mfma"):
                    v = dict(shape=shape, K=K, d=3, r=r, dtype=dt, T=T, path=path, dims=(n, n, n),
                             steps=50, boundary="periodic")
                    row[path] = measure(stl, v, x, w, 2, 1)
                name = f"{shape}-3d{r}r-{dt}-T{T}"
                res[name] = row
                log(f"{name}: " + ", ".join(f"{k} {v_.get('gst', float('nan')):.1f}" for k, v_ in row.items()))
        del x
        torch.cuda.empty_cache()
    return res


def measured_ceilings(stl):
    """Microbenchmarked ceilings per dtype (the model's second column): HBM
    copy bandwidth, FMA chains on the vector units (float32 with vector
    operands, as the kernels use), dense matrix-core rates; the sparse
    matrix rate is taken as twice the dense one (not measured)."""
    m = {k: stl.microbench(k) for k in ("copy", "fma_f64", "fma_f32_vgpr", "mfma_f64", "mfma_f32", "mfma_bf16")}
    hw = {}
    for dt, valu, mfma in (("f64", "fma_f64", "mfma_f64"), ("f32", "fma_f32_vgpr", "mfma_f32"),
                           ("bf16", "fma_f32_vgpr", "mfma_bf16"), ("f16", "fma_f32_vgpr", "mfma_bf16"),
                           ("bf16x3", "fma_f32_vgpr", "mfma_bf16")):
        hw[dt] = dict(BB=m["copy"], PP_valu=m[valu], PP_mfma=m[mfma], PP_mfma_sparse=2 * m[mfma])
    log("measured ceilings: " + ", ".join(f"{k} {v / 1e12:.2f}" for k, v in m.items()))
    return dict(raw=m, per_dtype=hw)


def parse_case(name):
    """(shape, d, r, dtype, T) of a variant name such as box-2d3r-f64-T2."""
    m = re.match(r"(box|star)-(\d)d(\d)r-(\w+)-T(\d+)", name)
    return (m.group(1), int(m.group(2)), int(m.group(3)), m.group(4), int(m.group(5))) if m else None


def predicted_with(stl, hw, name):
    c = parse_case(name)
    if not c or not hw:
        return None
    shape, d, r, dt, T = c
    m = stl.model_predict(shape, d, r, T, dt, hw=hw["per_dtype"][dt])
    return {-1: "valu", 0: "tie", 1: "mfma"}[m["winner"]]


def model_check(c2, c3):
    rows = []
    pairs = {}
    for name, r in c2.items():
        if "gst" not in r:
            continue
        key = name.rsplit("-", 1)[0]
        pairs.setdefault(key, {})[r["path"]] = r
    for key, row in list(pairs.items()) + [(k, v) for k, v in c3.items()]:
        if "gst" not in row.get("valu", {}) or "gst" not in row.get("mfma", {}):
            continue
        pred = {-1: "valu", 0: "tie", 1: "mfma"}[row["valu"]["predicted_winner"]]
        ratio = row["mfma"]["gst"] / row["valu"]["gst"]
        rows.append(dict(case=key, predicted=pred, measured=verdict(ratio), ratio=ratio,
                         scenario=row["valu"]["scenario"], valu_gst=row["valu"]["gst"],
                         mfma_gst=row["mfma"]["gst"], S=row["mfma"]["S"], alpha=row["mfma"]["alpha"]))
    agree = sum(r["predicted"] == r["measured"] for r in rows)
    return dict(cases=rows, agree=agree, total=len(rows))


# ---------------------------------------------------------------- paper's cases
# The six representative cases of the paper's Table 3 (pattern, fusion depth,
# type), run on MI355X at the paper's domain sizes (10240^2, 1024^3; Sec.
# "Experiments"): both paths at that depth, the model's predicted winner next
# to the measured one.  The A100 GStencil/s the paper prints (CUDA-core
# baseline, Tensor-Core implementation) are quoted as context only.
PAPER_CASES = [
    ("1", "box", 2, 1, 3, "f64", (260.90, 190.14)),
    ("2", "box", 2, 3, 1, "f64", (64.05, 63.33)),
    ("3", "box", 2, 1, 7, "f32", (318.31, 1002.94)),
    ("4", "box", 2, 7, 1, "f32", (50.35, 143.28)),
    ("5", "box", 3, 1, 3, "f64", (37.74, 24.63)),
    ("6", "box", 3, 1, 7, "f32", (71.23, 51.13)),
]


def section_cases(stl, args):
    import torch

    import stencil_inputs as si

    out = {}
    for case, shape, d, r, T, dt, a100 in PAPER_CASES:
        n = 10240 if d == 2 else 1024
        dims = (n,) * d
        K = (2 * r + 1) ** d
        w = si.normalised_weights(K, seed=si.weight_seed(6, int(case)))
        g = torch.Generator(device="cuda")
        g.manual_seed(si.data_seed(6, int(case)))
        x = torch.rand(dims, generator=g, device="cuda", dtype=torch.float64).to(stl.torch_dtype(dt))
        row = dict(pattern=f"{shape}-{d}d{r}r", T=T, dtype=dt, dims=list(dims), a100_gst=list(a100))
        m = stl.model_predict(shape, d, r, T, dt)
        row["predicted"] = {-1: "valu", 0: "tie", 1: "mfma"}[m["winner"]]
        row["predicted_ratio"] = m["ratio"]
        row["scenario"] = m["scenario"]
        for path in ("valu", "mfma"):
            Tp = T
            if not stl.kernel_available(path, dt, shape, d, r, T):
                if path == "mfma":
                    row[path] = dict(error=f"no MFMA kernel with composite radius {r * T} in {d}D")
                    continue
                # deepest fused VALU depth this pattern has
                Tp = max(t for t in range(1, T + 1) if stl.kernel_available(path, dt, shape, d, r, t))
            v = dict(shape=shape, K=K, d=d, r=r, dtype=dt, T=Tp, path=path, dims=dims, steps=4 * Tp,
                     boundary="periodic")
            res = measure(stl, v, x, w, 3, 1)
            res["T_run"] = Tp
            row[path] = res
        if "gst" in row["valu"] and "gst" in row.get("mfma", {}):
            row["measured"] = verdict(row["mfma"]["gst"] / row["valu"]["gst"])
            row["measured_ratio"] = row["mfma"]["gst"] / row["valu"]["gst"]
        out[case] = row
        log(f"case {case} {row['pattern']} T{T} {dt}: valu {row['valu'].get('gst', float('nan')):.1f} "
            f"(T={row['valu'].get('T_run')}), mfma {row.get('mfma', {}).get('gst', float('nan')):.1f}; "
            f"predicted {row['predicted']}, measured {row.get('measured', '-')}")
        del x
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------- the paper's benchmark grid
# Sec. "Evaluation Setup" (Benchmarks): box and star patterns of radius 1, 3
# and 7 on 10240^2 grids and of radius 1 on 1024^3 grids, double and float.
# Each pattern runs one step per pass and fused (radius 1: the paper's depths
# 3 and 7 in 2D, 3 in 3D; radius 3: 2; radius 7: none) on both paths, with
# the model's predicted winner next to the measured one.
GRID = ([(shape, 2, 1, T) for shape in ("box", "star") for T in (1, 3, 7)]
        + [(shape, 2, 3, T) for shape in ("box", "star") for T in (1, 2)]
        + [(shape, 2, 7, 1) for shape in ("box", "star")]
        + [(shape, 3, 1, T) for shape in ("box", "star") for T in (1, 3)])


def section_grid(stl, args):
    import torch

    import stencil_inputs as si

    out = {}
    xs = {}
    for shape, d, r, T in GRID:
        n = 10240 if d == 2 else 1024
        dims = (n,) * d
        K = (2 * r + 1) ** d if shape == "box" else 2 * d * r + 1
        w = si.normalised_weights(K, seed=si.weight_seed(7, 100 * d + 10 * r + (shape == "box")))
        for dt in ("f64", "f32"):
            if (d, dt) not in xs:
                xs.clear()
                torch.cuda.empty_cache()
                g = torch.Generator(device="cuda")
                g.manual_seed(si.data_seed(7, d))
                xs[(d, dt)] = torch.rand(dims, generator=g, device="cuda", dtype=torch.float64).to(
                    stl.torch_dtype(dt))
            x = xs[(d, dt)]
            m = stl.model_predict(shape, d, r, T, dt)
            row = dict(predicted={-1: "valu", 0: "tie", 1: "mfma"}[m["winner"]], predicted_ratio=m["ratio"])
            for path in ("valu", "mfma"):
                if not stl.kernel_available(path, dt, shape, d, r, T):
                    row[path] = dict(error="no kernel fuses this depth")
                    continue
                v = dict(shape=shape, K=K, d=d, r=r, dtype=dt, T=T, path=path, dims=dims, steps=4 * T,
                         boundary="periodic")
                res = measure(stl, v, x, w, 3, 1)
                row[path] = {k: res[k] for k in ("gst", "roofline", "predicted_gst") if k in res} or res
            if "gst" in row.get("valu", {}) and "gst" in row.get("mfma", {}):
                row["measured_ratio"] = row["mfma"]["gst"] / row["valu"]["gst"]
                row["measured"] = verdict(row["measured_ratio"])
            name = f"{shape}-{d}d{r}r-{dt}-T{T}"
            out[name] = row
            log(f"grid {name}: valu {row.get('valu', {}).get('gst', float('nan')):.1f}, mfma "
                f"{row.get('mfma', {}).get('gst', float('nan')):.1f}; predicted {row['predicted']}, "
                f"measured {row.get('measured', '-')}")
    xs.clear()
    torch.cuda.empty_cache()
    rows = [r for r in out.values() if "measured" in r]
    return dict(cases=out, agree=sum(r["predicted"] == r["measured"] for r in rows), total=len(rows))


# ---------------------------------------------------------------- sequential vs kernel fusion on MFMA
# Kernel fusion (the composite of T steps, redundancy alpha) against
# sequential-step fusion (T single-step band products, alpha = 1, the halo
# recomputed each step), both on the matrix cores, with the model's
# executed work per point for each (C_mfma, C_mfma_seq) and its prediction.
SEQ_CASES = ([("box", 3, T, dt, 8192, "dirichlet") for dt in ("f64", "f32") for T in (2, 4)]
             + [("star", 3, T, dt, 8192, "dirichlet") for dt in ("f64", "f32") for T in (2, 4)]
             + [("box", 2, 4, "bf16", 16384, "periodic")])


def section_seq(stl, args):
    import torch

    import stencil_inputs as si

    out = {}
    xs = {}
    for shape, r, T, dt, n, bnd in SEQ_CASES:
        K = (2 * r + 1) ** 2 if shape == "box" else 4 * r + 1
        w = si.normalised_weights(K, seed=si.weight_seed(2, 0 if shape == "box" else 1))
        if (n, dt) not in xs:
            xs.clear()
            torch.cuda.empty_cache()
            xs[(n, dt)] = si.round_to(si.uniform_grid((n, n), seed=si.data_seed(2, 0)), dt)[1].to("cuda")
        x = xs[(n, dt)]
        m = stl.model_predict(shape, 2, r, T, dt)
        row = dict(C_kernel_fused=m["C_mfma"], C_sequential=m["C_mfma_seq"], model_gst_kernel_fused=m["gst_mfma"],
                   model_gst_sequential=m["gst_mfma_seq"])
        for path in ("mfma", "mfma_seq"):
            v = dict(shape=shape, K=K, d=2, r=r, dtype=dt, T=T, path=path, dims=(n, n), steps=100,
                     boundary=bnd)
            res = measure(stl, v, x, w, 3, 1)
            row[path] = res.get("gst", res.get("error"))
        name = f"{shape}-2d{r}r-{dt}-T{T}-{n}"
        out[name] = row
        log(f"seq {name}: kernel-fused {row['mfma']}, sequential {row['mfma_seq']} GSt/s; model "
            f"{row['model_gst_kernel_fused']:.0f} vs {row['model_gst_sequential']:.0f} "
            f"(executed flop/point/pass {row['C_kernel_fused']:.0f} vs {row['C_sequential']:.0f})")
    xs.clear()
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------- dense vs 2:4 sparse matrix units
# The paper's Table 4 compares one kernel on dense and on sparse Tensor Cores
# (Box-2D1R fused 7 deep, float, Sec. "Further Acceleration with Sparse
# Hardware"); gfx950's sparse instructions take 16-bit operands, so the MI355X
# analogue runs bf16 storage with float32 accumulation, periodic grids, on the
# dense band layout and on the 2:4 layout, next to the model's prediction
# for each (sparse: the doubled matrix peak).
SPARSE_CASES = [("box", 1, 7, 10240), ("box", 2, 3, 16384), ("box", 3, 2, 8192), ("star", 3, 2, 8192)]


def section_sparse(stl, args):
    import torch

    import stencil_inputs as si

    out = {}
    for shape, r, T, n in SPARSE_CASES:
        K = (2 * r + 1) ** 2 if shape == "box" else 4 * r + 1
        w = si.normalised_weights(K, seed=si.weight_seed(6, 10 + r * 10 + T))
        g = torch.Generator(device="cuda")
        g.manual_seed(si.data_seed(6, 10 + r * 10 + T))
        x = torch.rand((n, n), generator=g, device="cuda", dtype=torch.float64).to(torch.bfloat16)
        row = {}
        for path in ("mfma", "mfma_sparse"):
            v = dict(shape=shape, K=K, d=2, r=r, dtype="bf16", T=T, path=path, dims=(n, n), steps=4 * T,
                     boundary="periodic")
            res = measure(stl, v, x, w, 3, 1)
            m = stl.model_predict(shape, 2, r, T, "bf16", sparse=(path == "mfma_sparse"))
            if "gst" in res:
                res["model_gst"] = m["gst_mfma"]
                res["model_S"] = m["S"]
            row[path] = res
        name = f"{shape}-2d{r}r-bf16-T{T}-{n}"
        if "gst" in row["mfma"] and "gst" in row["mfma_sparse"]:
            row["speedup"] = row["mfma_sparse"]["gst"] / row["mfma"]["gst"]
            row["model_speedup"] = row["mfma_sparse"]["model_gst"] / row["mfma"]["model_gst"]
        out[name] = row
        log(f"sparse {name}: dense {row['mfma'].get('gst', float('nan')):.1f}, sparse "
            f"{row['mfma_sparse'].get('gst', float('nan')):.1f} GSt/s (measured x{row.get('speedup', float('nan')):.2f},"
            f" model x{row.get('model_speedup', float('nan')):.2f})")
        del x
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------- 16384^2 precision workload
def section_c4(stl, args):
    import numpy as np
    import torch

    import stencil_inputs as si

    n = 16384
    u0 = si.smooth_grid((n, n), seed=si.data_seed(4, 0))
    w = si.normalised_weights(25, seed=si.weight_seed(4, 0))
    npts = n * n

    def sweep(dtype, path, T, x0):
        p = stl.Plan("box", 2, 2, w, (n, n), T=T, dtype=dtype, path=path, boundary="periodic")
        x = x0.clone()
        y = torch.empty_like(x)
        snaps, ms_total = [], 0.0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(10):
            e0.record()
            p.run(x, y, 100)
            e1.record()
            torch.cuda.synchronize()
            ms_total += e0.elapsed_time(e1)
            x, y = y, x
            snaps.append(x)
            x = x.clone()
        p.close()
        return snaps, ms_total

    golden = load_precision_windows(w)
    ref0 = torch.from_numpy(u0).to("cuda")
    ref_snaps, ref_ms = sweep("f64", "valu", 2, ref0)
    log(f"f64 reference: {npts * 1000 / (ref_ms * 1e-3) / 1e9:.1f} GSt/s")
    out = {"reference": dict(dtype="f64", path="valu", T=2, gst=npts * 1000 / (ref_ms * 1e-3) / 1e9)}
    if golden:
        out["reference"]["oracle_window_err_1000"] = window_err(ref_snaps[-1], golden, "f64")
    modes = [("bf16", "mfma", 4), ("f16", "mfma", 4), ("bf16x3", "mfma", 4), ("bf16", "mfma", 2),
             ("bf16", "valu", 2), ("f16", "valu", 2), ("f32", "valu", 2), ("f32", "mfma", 4)]
    for dt, path, T in modes:
        x0 = si.round_to(u0, dt)[1].to("cuda")
        try:
            snaps, ms = sweep(dt, path, T, x0)
        except stl.StencilError as e:
            out[f"{dt}-{path}-T{T}"] = dict(error=str(e))
            continue
        errs = []
        for k, (s_, rsnap) in enumerate(zip(snaps, ref_snaps)):
            d = (s_.to(torch.float64) - rsnap)
            errs.append(float(d.abs().max() / rsnap.abs().max()))
            del d
        m = stl.model_predict("box", 2, 2, T, dt)
        row = dict(gst=npts * 1000 / (ms * 1e-3) / 1e9, err_every_100=errs,
                   predicted_winner=m["winner"], scenario=m["scenario"],
                   predicted_gst=m["gst_valu"] if path == "valu" else m["gst_mfma"])
        if golden:
            # end-to-end: oracle on the float64 data; arithmetic: oracle on
            # the storage-rounded data (both after 1000 steps, on the stored
            # window), relative to the window's max |u|
            row["oracle_e2e_1000"] = window_err(snaps[-1], golden, "f64")
            row["oracle_arith_1000"] = window_err(snaps[-1], golden,
                                                  {"bf16x3": "f32"}.get(dt, dt))
        out[f"{dt}-{path}-T{T}"] = row
        log(f"{dt}-{path}-T{T}: {row['gst']:.1f} GSt/s, err@1000 vs f64 sweep {errs[-1]:.2e}"
            + (f", vs oracle window: end-to-end {row['oracle_e2e_1000']:.2e}, arithmetic "
               f"{row['oracle_arith_1000']:.2e}" if golden else ""))
        del snaps, x0
        torch.cuda.empty_cache()
    del ref_snaps, ref0
    torch.cuda.empty_cache()
    return out


def load_precision_windows(w):
    """FP64 oracle values of the precision workload after 1000 steps on one
    window (written by tests/golden/make_precision_windows.py from the
    oracle), or None if absent or made for other weights."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", "precision_windows_16384.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    if not np.array_equal(np.asarray(g["weights"]), w):
        return None
    return g


def window_err(snap, golden, key):
    import numpy as np

    lo, hi = golden["lo"], golden["hi"]
    got = snap[lo[0]:hi[0], lo[1]:hi[1]].double().cpu().numpy()
    ref = np.asarray(golden["windows"][key]["values"])
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


# ---------------------------------------------------------------- served stream
def _served_jobs(stl, trace, scale_arrivals=1.0):
    import torch

    import stencil_inputs as si
    from paper_2603_00477_amd.serve import Job

    jobs = []
    for t in trace:
        K = (2 * t["r"] + 1) ** t["d"] if t["shape"] == "box" else 2 * t["d"] * t["r"] + 1
        w = si.normalised_weights(K, t["weight_seed"])
        seed = t["data_seed"]

        def gen(device, dims=t["dims"], seed=seed):
            g = torch.Generator(device=device)
            g.manual_seed(seed)
            return torch.rand(dims, generator=g, device=device, dtype=torch.float32)

        jobs.append(Job(t["shape"], t["d"], t["r"], w, t["dims"], t["steps"], dtype="f32",
                        boundary=t["boundary"], data=gen, arrival=t["arrival"] * scale_arrivals,
                        id=t["id"]))
    return jobs


def _serve(ex, jobs, t0, budget):
    """Submit each job at its arrival time to a fresh server; returns timing
    records (outputs are dropped as soon as they arrive)."""
    import time as _t

    from paper_2603_00477_amd.serve import StencilServer

    srv = StencilServer(ex, hbm_budget=budget).start()
    futs = []
    for j in jobs:
        now = _t.perf_counter() - t0
        if j.arrival > now:
            _t.sleep(j.arrival - now)
        j.arrival = None
        f = srv.submit(j)
        f.add_done_callback(lambda f: setattr(f.result(), "output", None) if not f.exception() else None)
        futs.append(f)
    for f in futs:
        f.result()
    srv.stop()
    return srv.done, srv.rounds


def section_serving(stl, args):
    import torch

    import stencil_inputs as si
    from paper_2603_00477_amd.serve import GpuExecutor, latency_stats, run_fifo

    budget = 32 << 30
    trace = si.served_trace(args.jobs, seed=5000, rate_per_s=1.0)
    work = sum(math.prod(t["dims"]) * t["steps"] for t in trace)
    ex = GpuExecutor()
    out = dict(jobs=len(trace), point_steps=work, hbm_budget=budget)
    # autotune every problem class once (first job of each class) before the
    # timed legs, so that both legs run the same tuned plans
    t0 = time.perf_counter()
    seen = set()
    for j in _served_jobs(stl, trace, scale_arrivals=0.0):
        key = ex.problem_class(j)
        if key in seen:
            continue
        seen.add(key)
        ex.release(ex.prepare(j))
    torch.cuda.synchronize()
    out["tuned_classes"] = len(ex.choices)
    out["tuning_s"] = time.perf_counter() - t0
    paths = [c[0] for c in ex.choices.values()]
    out["tuned_mfma_classes"] = sum(1 for pth in paths if pth == 2)
    out["tuned_T_histogram"] = {str(T): sum(1 for c in ex.choices.values() if c[1] == T) for T in range(1, 5)}
    log(f"serving: tuned {len(ex.choices)} problem classes in {out['tuning_s']:.1f} s "
        f"(T histogram {out['tuned_T_histogram']}, MFMA classes {out['tuned_mfma_classes']})")
    # capacity: every job available at t = 0
    for mode in ("fifo", "served"):
        jobs = _served_jobs(stl, trace, scale_arrivals=0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "fifo":
            done = run_fifo(ex, jobs, t0=t0, keep_outputs=False)
        else:
            done, rounds = _serve(ex, jobs, t0, budget)
        span = max(d.finished for d in done) - t0
        out[f"{mode}_capacity"] = dict(jobs_per_s=len(jobs) / span, gst=work / span / 1e9, makespan_s=span)
        log(f"serving capacity {mode}: {len(jobs) / span:.1f} jobs/s, {work / span / 1e9:.1f} GSt/s")
        torch.cuda.empty_cache()
    # Poisson arrivals at 0.8 x the one-plan-per-call capacity (trace drawn at
    # rate 1/s, arrival times rescaled)
    rate = 0.8 * out["fifo_capacity"]["jobs_per_s"]
    out["arrival_rate_jobs_per_s"] = rate
    for mode in ("served", "fifo"):
        jobs = _served_jobs(stl, trace, scale_arrivals=1.0 / rate)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "fifo":
            done = run_fifo(ex, jobs, t0=t0, keep_outputs=False)
        else:
            done, rounds = _serve(ex, jobs, t0, budget)
            out["rounds"] = rounds
        span = max(d.finished for d in done) - t0
        st = latency_stats(done)
        out[mode] = dict(p50_ms=st["p50_ms"], p99_ms=st["p99_ms"], mean_ms=st["mean_ms"],
                         gst=work / span / 1e9, makespan_s=span)
        log(f"serving {mode} at 0.8 load: p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms, "
            f"{work / span / 1e9:.1f} GSt/s")
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------- CPU baseline / traffic
def cpu_baseline(n, budget_s):
    import stencil_inputs as si
    from oracle import core

    w = si.normalised_weights(49, seed=si.weight_seed(2, 0))
    u0 = si.uniform_grid((n, n), seed=si.data_seed(2, 0))
    threads = core.max_threads()
    t0 = time.perf_counter()
    core.run("box", 2, 3, w, u0, 1, "dirichlet", 0.0)
    one = time.perf_counter() - t0
    k = max(1, min(20, int(budget_s / max(one, 1e-3)) - 1))
    t0 = time.perf_counter()
    core.run("box", 2, 3, w, u0, k, "dirichlet", 0.0)
    dt = time.perf_counter() - t0
    return dict(value=n * n * k / dt / 1e9, unit="GStencil/s", cores=threads, kind="oracle",
                sample=f"Box-2D3R f64 {n}x{n}, {k} time steps (of 100), zero Dirichlet halo",
                cpu_model=cpu_model(), nproc=os.cpu_count(),
                affinity=len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _smi_clocks():
    """Current shader (sclk) and memory (mclk) clocks in MHz from rocm-smi,
    or None."""
    import subprocess

    try:
        p = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True,
                           timeout=30)
        data = json.loads(p.stdout)
    except Exception:
        return None
    out = {}
    for card in data.values():
        if not isinstance(card, dict):
            continue
        for k, v in card.items():
            m = re.search(r"(\d+)\s*Mhz", str(v), re.I)
            for name in ("sclk", "mclk", "fclk", "socclk"):
                if m and k.lower().startswith(name) and "speed" in k.lower():
                    out[f"{name}_mhz"] = int(m.group(1))
        break
    return out or None


def clocks_under_load(busy):
    """Clocks sampled while `busy()` keeps the GPU working (the reading is
    taken in another thread during about two seconds of work)."""
    import threading

    box = {}
    th = threading.Thread(target=lambda: box.setdefault("c", _smi_clocks()))
    t0 = time.perf_counter()
    th.start()
    while th.is_alive() and time.perf_counter() - t0 < 30:
        busy()
    th.join()
    return box.get("c")


def source_hash():
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def recorded_traffic(variant):
    """HBM bytes per launch recorded under profiles/ for `variant`, if the
    kernel sources still hash to the recorded value."""
    path = os.path.join(ROOT, "profiles", "traffic_valu2d_box2d3r_8192.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"sources_sha1:\s*([0-9a-f]+)", txt)
    if not m or m.group(1) != source_hash():
        return None
    m = re.search(rf"^\|\s*{re.escape(variant)}\s*\|\s*([0-9.eE+]+)\s*\|", txt, re.M)
    return float(m.group(1)) if m else None


# ---------------------------------------------------------------- output
def _r(x, nd=1):
    return None if x is None else round(float(x), nd)


def _sig(x, nd=3):
    return None if x is None else float(f"{float(x):.{nd}g}")


def summaries(variants, mcheck, precision, serving, cases, sparse=None, grid=None, seq=None):
    """One-line summaries of every section for the JSON line (the full
    per-variant detail goes to --json-out / stderr)."""
    out = {}
    if variants:
        out["variants_gst"] = {k.replace("-2d3r", ""): _r(r["gst"]) for k, r in variants.items()}
    if mcheck:
        out["model_check"] = f"{mcheck['agree']}/{mcheck['total']}"
        if "agree_measured_ceilings" in mcheck:
            out["model_check_measured_ceilings"] = f"{mcheck['agree_measured_ceilings']}/{mcheck['total']}"
    if precision:
        out["precision"] = {k: [_r(v["gst"]), _sig(v.get("oracle_e2e_1000", v["err_every_100"][-1])),
                                _sig(v.get("oracle_arith_1000"))]
                            for k, v in precision.items() if k != "reference" and "gst" in v}
    if serving:
        out["serving"] = {
            "served": [_r(serving["served"]["p50_ms"], 2), _r(serving["served"]["p99_ms"], 2),
                       _r(serving["served"]["gst"])],
            "fifo": [_r(serving["fifo"]["p50_ms"], 2), _r(serving["fifo"]["p99_ms"], 2),
                     _r(serving["fifo"]["gst"])],
            "capacity_gst": [_r(serving["served_capacity"]["gst"]), _r(serving["fifo_capacity"]["gst"])]}
    if cases:
        out["paper_cases"] = {k: [_r(c.get("valu", {}).get("gst")), _r(c.get("mfma", {}).get("gst")),
                                  c["predicted"], c.get("measured")] for k, c in cases.items()}
    if grid:
        out["grid_model_check"] = f"{grid['agree']}/{grid['total']}"
        if "agree_measured_ceilings" in grid:
            out["grid_model_check_measured_ceilings"] = f"{grid['agree_measured_ceilings']}/{grid['total']}"
    if seq:
        out["sequential"] = {k.replace("-2d", "").replace("-8192", "").replace("-16384", ""):
                             [_r(c["mfma"]) if isinstance(c["mfma"], float) else None,
                              _r(c["mfma_seq"]) if isinstance(c["mfma_seq"], float) else None]
                             for k, c in seq.items()}
    if sparse:
        out["sparse"] = {k: [_r(c.get("mfma", {}).get("gst")), _r(c.get("mfma_sparse", {}).get("gst")),
                             _r(c.get("model_speedup"), 2)] for k, c in sparse.items()}
    return out


SUMMARY_KEYS = {
    "variants_gst": "GStencil/s per 8192^2 variant (shape-dtype-T-path)",
    "precision": "16384^2 Box-2D2R, 1000 steps: [GStencil/s, end-to-end error, arithmetic error] "
                 "(relative, against the FP64 oracle on a window after 1000 steps)",
    "serving": "served stream: [p50 ms, p99 ms, GStencil/s] at 0.8 load; capacity_gst [served, fifo]",
    "paper_cases": "Table 3 cases at 10240^2 / 1024^3: [VALU, MFMA GStencil/s, predicted, measured]",
    "sparse": "Table 4 analogue, bf16 periodic: [dense MFMA, 2:4 sparse MFMA GStencil/s, model sparse/dense]",
    "sequential": "MFMA [kernel fusion, sequential-step fusion] GStencil/s (100 steps; 8192^2 Dirichlet, "
                  "bf16 16384^2 periodic)",
    "grid_model_check": "the paper's benchmark grid (box/star r 1,3,7 at 10240^2, r 1 at 1024^3, f64/f32, "
                        "one-step and fused passes): predicted winner = measured / cases with both paths",
}


def compact_line(args, head_name, head, hv, roof, cpu, clocks, summ):
    """The JSON line on stdout (kept under 4 KB)."""
    line = {
        "metric": "GStencil/s",
        "value": _r(head.get("gst"), 2),
        "unit": "GStencil/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": _r(head.get("ms_per_sweep"), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": hv["dtype"] if hv else None,
        "data": "synthetic",
        "config": {"workload": (f"Box-2D3R {args.n}x{args.n} {hv['dtype']}, {args.time_steps} time steps "
                                f"per step, zero Dirichlet halo, T={hv['T']}, {head['path']} path")
                   if hv else None,
                   "step": f"one sweep of {args.time_steps} time steps over the whole grid"},
        "roofline": ({k: (_sig(v, 4) if isinstance(v, float) else v) for k, v in roof.items()}
                     if roof else None),
        "cpu_baseline": ({k: (_sig(v, 4) if isinstance(v, float) else v) for k, v in cpu.items()}
                         if cpu else None),
        "clocks": clocks,
        "summary": summ,
    }
    return json.dumps(line, separators=(",", ":"))


# ---------------------------------------------------------------- main
def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the stencil library has no multi-GPU path "
              "(a grid would shard as slabs along its slowest axis with an r*T-deep halo "
              "exchange per pass); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2603_00477_amd as stl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stl.lib()
    sections = set(args.sections.split(","))
    c2 = section_c2(stl, args) if "c2" in sections else {}
    ok = {k: r for k, r in c2.items() if "gst" in r}
    box64 = {k: r for k, r in ok.items() if k.startswith("box-2d3r-f64")}
    pool = box64 or ok
    head_name = max(pool, key=lambda k: pool[k]["gst"]) if pool else None
    hv = next((v for v in headline_variants(args.n, args.time_steps) if v["name"] == head_name), None)
    clocks = None
    if hv and not args.no_clocks:
        clocks = headline_clocks(stl, args, hv)
    c3 = section_c3(stl, args) if "c3" in sections else {}
    c4 = section_c4(stl, args) if "c4" in sections else None
    c5 = section_serving(stl, args) if "c5" in sections else None
    cases = section_cases(stl, args) if "cases" in sections else None
    sparse = section_sparse(stl, args) if "sparse" in sections else None
    grid = section_grid(stl, args) if "grid" in sections else None
    seq = section_seq(stl, args) if "seq" in sections else None
    cpu = None if args.no_cpu or not head_name else cpu_baseline(args.n, args.cpu_seconds)
    head = ok.get(head_name, {})
    roof = dict(head.get("roofline", {}))
    if roof:
        roof["traffic"] = recorded_traffic(head_name)
    mcheck = model_check(c2, c3) if (c2 or c3) else None
    ceil = None
    if mcheck or grid:
        try:
            ceil = measured_ceilings(stl)
        except Exception as e:  # the datasheet column stands alone then
            log(f"measured ceilings unavailable: {e}")
    if ceil:
        for rows in ([mcheck["cases"]] if mcheck else []) + ([list(grid["cases"].items())] if grid else []):
            for item in rows:
                name, row = (item["case"], item) if isinstance(item, dict) else item
                if "measured" not in row:
                    continue
                row["predicted_measured_ceilings"] = predicted_with(stl, ceil, name)
        if mcheck:
            mcheck["agree_measured_ceilings"] = sum(r.get("predicted_measured_ceilings") == r["measured"]
                                                    for r in mcheck["cases"])
        if grid:
            rows = [r for r in grid["cases"].values() if "measured" in r]
            grid["agree_measured_ceilings"] = sum(r.get("predicted_measured_ceilings") == r["measured"]
                                                  for r in rows)
    detail = {
        "headline": head_name, "roofline": roof or None, "cpu_baseline": cpu, "clocks": clocks,
        "variants": ok, "model_check": mcheck, "ceilings": ceil, "precision": c4, "serving": c5,
        "paper_cases": cases,
        "sparse": sparse, "grid": grid, "sequential": seq,
        "summary_keys": SUMMARY_KEYS,
    }
    s = json.dumps(detail)
    if args.json_out:
        with open(args.json_out, "w") as f:
            f.write(s + "\n")
    else:
        print("# detail " + s, file=sys.stderr, flush=True)
    print(compact_line(args, head_name, head, hv, roof, cpu, clocks,
                       summaries(ok, mcheck, c4, c5, cases, sparse, grid, seq)), flush=True)


def headline_clocks(stl, args, hv):
    """sclk / mclk while the headline plan runs."""
    import torch

    import stencil_inputs as si

    n = args.n
    x = torch.rand((n, n), device="cuda", dtype=stl.torch_dtype(hv["dtype"]))
    y = torch.empty_like(x)
    w = si.normalised_weights(hv["K"], seed=si.weight_seed(2, 0))
    p = stl.Plan(hv["shape"], 2, hv["r"], w, (n, n), T=hv["T"], dtype=hv["dtype"], path=hv["path"])

    def busy():
        p.run(x, y, args.time_steps)
        torch.cuda.synchronize()

    c = clocks_under_load(busy)
    p.close()
    log(f"clocks under load: {c}")
    return c


if __name__ == "__main__":
    main()
