"""Counter validation of the roofline model (measured C, M, I and S).

Two commands:

  python -m paper_2603_00477_amd.counters run [--n2 N] [--n3 N] [--set model|ai_t|p16]
      Runs one pass (T fused steps) of each listed variant on the GPU, two
      times, so that a rocprofv3 counter pass records every kernel.  Prints a
      JSON line per variant with the grid size and the model's C, M, I.

  python -m paper_2603_00477_amd.counters report FETCH.csv WRITE.csv SQ.csv RUN.jsonl
      Reads the rocprofv3 counter CSVs of three runs of `run` (FETCH_SIZE,
      WRITE_SIZE, and the SQ instruction counters) plus the JSON lines `run`
      printed, and writes a markdown table: per variant, the model's C, M, I
      next to the measured ones, and for MFMA kernels the measured S.

Measured quantities, per grid point per pass (paper, Sec. "Verification of
Proposed Formulations": achieved work and achieved traffic against the
modelled C and M):
  M = (FETCH_SIZE * f_fetch + WRITE_SIZE * f_write) / points, with f_* the
      factor that maps the counter of a device copy of known size onto its
      bytes (both counters in KiB);
  C (VALU) = SQ_INSTS_VALU_FMA_{F64,F32} * 64 lanes * 2 / points;
  C (MFMA) = SQ_INSTS_VALU_MFMA_MOPS_* * 512 / points (executed flops);
  S (MFMA) = useful flops (2 K_T per point) / executed flops.
"""
from __future__ import annotations

import argparse
import csv
import json
import math
import sys

VARIANTS_2D = [(s, 3, T, dt, path) for s in ("box", "star") for dt in ("f64", "f32") for T in (1, 2, 4)
               for path in ("valu", "mfma")]
VARIANTS_3D = [(s, r, T, dt, path) for s, r in (("star", 2), ("box", 1)) for dt in ("f64", "f32")
               for T in (1, 2, 3) for path in ("valu", "mfma")]
VARIANTS_16 = [("box", 2, T, dt, "mfma") for dt in ("bf16", "f16", "bf16x3") for T in (1, 2, 4)]
# the 8192^2 vector-unit variants of the benchmark's first workload
VARIANTS_HEAD = [(s, 3, T, dt, "valu") for s in ("box", "star") for dt in ("f64", "f32") for T in (1, 2, 4)]
# arithmetic intensity against fusion depth on the vector units (paper,
# Sec. "Arithmetic Intensity Analysis": Box-2D1R and Star-2D1R, double)
VARIANTS_AI_T = [(s, 1, T, "f64", "valu") for s in ("box", "star") for T in range(1, 9)]


def _k(shape, d, r):
    return (2 * r + 1) ** d if shape == "box" else 2 * d * r + 1


def run(n2: int, n3: int, which: str = "model"):
    import torch

    import paper_2603_00477_amd as stl

    if which == "ai_t":
        todo = [(2, v) for v in VARIANTS_AI_T]
    elif which == "p16":
        todo = [(2, v) for v in VARIANTS_16]
    elif which == "head":
        todo = [(2, v) for v in VARIANTS_HEAD]
    elif which == "v3":
        todo = [(3, v) for v in VARIANTS_3D if v[4] == "valu"]
    else:
        todo = [(2, v) for v in VARIANTS_2D] + [(3, v) for v in VARIANTS_3D] + [(2, v) for v in VARIANTS_16]
    x_cache = {}
    for d, (shape, r, T, dt, path) in todo:
        dims = (n2, n2) if d == 2 else (n3, n3, n3)
        key = (d, dt)
        if key not in x_cache:
            g = torch.Generator(device="cuda")
            g.manual_seed(1234)
            x_cache[key] = torch.rand(dims, generator=g, device="cuda", dtype=torch.float64).to(
                stl.torch_dtype(dt))
        x = x_cache[key]
        K = _k(shape, d, r)
        w = [1.0 / K] * K
        try:
            p = stl.Plan(shape, d, r, w, dims, T=T, dtype=dt, path=path, boundary="periodic")
        except stl.StencilError as e:
            print(json.dumps(dict(variant=f"{shape}-{d}d{r}r-{dt}-T{T}-{path}", error=str(e))), flush=True)
            continue
        y = torch.empty_like(x)
        for _ in range(2):
            p.run(x, y, T)
        torch.cuda.synchronize()
        i = p.info()
        m = stl.model_predict(shape, d, r, T, dt)
        print(json.dumps(dict(variant=f"{shape}-{d}d{r}r-{dt}-T{T}-{path}", path=path, dtype=dt, T=T,
                              K=K, K_T=i["K_T"], points=math.prod(dims), S=i["S"], alpha=i["alpha"],
                              C_valu=m["C_valu"], C_mfma=m["C_mfma"], M=m["M"], I_valu=m["I_valu"],
                              I_mfma=m["I_mfma"], kernel_hint=("valu" if path == "valu" else "mfma"),
                              dims=list(dims))), flush=True)
        p.close()


def _load(path):
    """{kernel name: {dispatch id: {counter: value}}}."""
    by = {}
    for r in csv.DictReader(open(path)):
        by.setdefault(r["Kernel_Name"], {}).setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = \
            float(r["Counter_Value"])
    return by


def _stencil_kernels(by):
    """Stencil kernel names in order of first dispatch, with averaged counters."""
    out = []
    for name, disp in by.items():
        if "stl::" not in name or not any(k in name for k in ("valu", "mfma", "fused3d")):
            continue
        first = min(disp)
        avg = {}
        for vals in disp.values():
            for c, v in vals.items():
                avg[c] = avg.get(c, 0.0) + v / len(disp)
        out.append((first, name, avg))
    out.sort()
    return [(n, a) for _, n, a in out]


def report(fetch_csv, write_csv, sq_csv, run_jsonl, f_fetch=2.0, f_write=1.0, out=sys.stdout):
    runs = [json.loads(l) for l in open(run_jsonl) if l.strip().startswith("{")]
    runs = [r for r in runs if "error" not in r]
    F = _stencil_kernels(_load(fetch_csv))
    Wr = _stencil_kernels(_load(write_csv))
    Q = _stencil_kernels(_load(sq_csv))
    if not (len(F) == len(Wr) == len(Q) == len(runs)):
        raise SystemExit(f"kernel/variant count mismatch: {len(F)} {len(Wr)} {len(Q)} {len(runs)}")
    print("| variant | C model | C meas (dC) | M model | M meas (dM) | I model | I meas | S model | S meas |",
          file=out)
    print("|---|---|---|---|---|---|---|---|---|", file=out)
    rows = []
    for r, (fn, fv), (wn, wv), (qn, qv) in zip(runs, F, Wr, Q):
        pts = r["points"]
        M = (fv["FETCH_SIZE"] * f_fetch + wv["WRITE_SIZE"] * f_write) * 1024.0 / pts
        if r["path"] == "valu":
            fma = qv.get("SQ_INSTS_VALU_FMA_F64", 0.0) + qv.get("SQ_INSTS_VALU_FMA_F32", 0.0)
            C = fma * 64 * 2 / pts
            Cm, Im = r["C_valu"], r["I_valu"]
            Sm, Sx = "", ""
        else:
            mops = sum(v for c, v in qv.items() if c.startswith("SQ_INSTS_VALU_MFMA_MOPS_"))
            C = mops * 512 / pts
            Cm, Im = r["C_mfma"], r["I_mfma"]
            useful = 2.0 * r["K_T"] * (3.0 if r["dtype"] == "bf16x3" else 1.0)
            Sm, Sx = f"{r['S']:.4f}", f"{useful / C:.4f}" if C > 0 else "n/a"
        row = dict(variant=r["variant"], C_model=Cm, C_meas=C, M_model=r["M"], M_meas=M, I_model=Im,
                   I_meas=C / M if M else float("nan"), S_model=Sm, S_meas=Sx)
        rows.append(row)
        print(f"| {r['variant']} | {Cm:.1f} | {C:.1f} ({100 * (C / Cm - 1):+.1f}%) | {r['M']:.2f} | "
              f"{M:.2f} ({100 * (M / r['M'] - 1):+.1f}%) | {Im:.2f} | {row['I_meas']:.2f} | {Sm} | {Sx} |",
              file=out)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--n2", type=int, default=4096)
    r.add_argument("--n3", type=int, default=256)
    r.add_argument("--set", default="model", choices=["model", "ai_t", "p16", "head", "v3"],
                   help="model: every 8192^2 / 512^3 / precision variant; ai_t: Box/Star-2D1R "
                        "float64 at T = 1..8; p16: the 16-bit and compensated MFMA variants only; "
                        "head: the 2D VALU variants of the first workload; v3: the 3D VALU variants")
    rep = sub.add_parser("report")
    rep.add_argument("fetch")
    rep.add_argument("write")
    rep.add_argument("sq")
    rep.add_argument("runs")
    rep.add_argument("--f-fetch", type=float, default=2.0,
                     help="bytes per FETCH_SIZE KiB of a device copy of known size / 1024")
    rep.add_argument("--f-write", type=float, default=1.0)
    a = ap.parse_args(argv)
    if a.cmd == "run":
        run(a.n2, a.n3, a.set)
    else:
        report(a.fetch, a.write, a.sq, a.runs, a.f_fetch, a.f_write)


if __name__ == "__main__":
    main()
