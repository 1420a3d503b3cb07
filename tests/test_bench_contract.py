"""Host-side pieces of bench.py: the roofline attribution of a launch, the
tie band of the winner verdict, the recorded-traffic lookup, and the
multi-GPU refusal.  No GPU needed."""
import json
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _info(path, T, K, S=1.0, alpha=1.0, gamma=1.0):
    return {"path": path, "T": T, "K": K, "S": S, "alpha": alpha, "gamma": gamma}


def test_valu_memory_bound_launch_reports_hbm_bytes():
    # Box-2D3R float64, T = 1: I = 49/8 = 6.1 flop/byte, below the 9.83 ridge
    npts = 8192 * 8192
    launch_ms = 0.25
    r = bench.roofline_for({"dtype": "f64"}, _info(1, 1, 49), launch_ms, npts)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    achieved = 16.0 * npts / (launch_ms * 1e-3)  # one read and one write of 8 bytes per point
    assert math.isclose(r["achieved"], achieved / 1e9)
    assert math.isclose(r["frac"], achieved / 8.0e12)


def test_valu_compute_bound_launch_reports_flops():
    # Box-2D3R float64, T = 2: I = 12.25 > 9.83 -> vector ALU, 2 K T flops per point
    npts = 8192 * 8192
    r = bench.roofline_for({"dtype": "f64"}, _info(1, 2, 49), 0.4, npts)
    assert r["bound"] == "alu" and r["peak"] == pytest.approx(78.6)
    assert math.isclose(r["achieved"], 2 * 49 * 2 * npts / 0.4e-3 / 1e12)
    # float32 takes its own ridge (157.3 / 8 = 19.7): T = 2 box r = 3 is above it
    r32 = bench.roofline_for({"dtype": "f32"}, _info(1, 2, 49), 0.2, npts)
    assert r32["bound"] == "alu" and r32["peak"] == pytest.approx(157.3)
    # ... and T = 1 (12.25 flop/byte) below it
    assert bench.roofline_for({"dtype": "f32"}, _info(1, 1, 49), 0.2, npts)["bound"] == "hbm"


def test_mfma_launch_counts_executed_work_against_the_matrix_peak():
    # float64 Box-2D3R T = 2 on the band layout: executed intensity
    # 2*49/8 * alpha/S = 12.25 * 1.72 / 0.464 = 45.5 flop/byte, above the 9.83 ridge
    npts = 8192 * 8192
    info = _info(2, 2, 49, S=0.4642857, alpha=169 / 98)
    r = bench.roofline_for({"dtype": "f64"}, info, 1.0, npts)
    assert r["bound"] == "mfma" and r["peak"] == pytest.approx(78.6)
    executed = 2 * 49 * 2 * npts * info["alpha"] / info["S"]
    assert math.isclose(r["achieved"], executed / 1e-3 / 1e12)
    # bf16 Box-2D2R T = 4: executed intensity 50 * 2.89 / 0.531 = 272 flop/byte stays below
    # the bf16 ridge (2516.6 / 8 = 314.6): the launch is attributed to HBM
    info16 = _info(2, 4, 25, S=0.53125, alpha=289 / 100)
    assert bench.roofline_for({"dtype": "bf16"}, info16, 1.0, 16384 * 16384)["bound"] == "hbm"


def test_verdict_tie_band():
    assert bench.verdict(1.16) == "mfma"
    assert bench.verdict(1.15) == "tie"
    assert bench.verdict(0.87) == "tie"
    assert bench.verdict(0.869) == "valu"


def test_recorded_traffic_requires_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # kernel sources copied so that the hash is computable in the fake root
    for f in bench.KERNEL_SOURCES:
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_bytes(open(os.path.join(ROOT, f), "rb").read())
    h = bench.source_hash()
    body = "| box-2d3r-f64-T2-valu | 1.133e+09 | 16.88 |\n"
    (prof / "traffic_valu2d_box2d3r_8192.md").write_text(f"sources_sha1: {h}\n\n" + body)
    assert bench.recorded_traffic("box-2d3r-f64-T2-valu") == pytest.approx(1.133e9)
    assert bench.recorded_traffic("box-2d3r-f64-T1-valu") is None
    (prof / "traffic_valu2d_box2d3r_8192.md").write_text("sources_sha1: 000000000000\n\n" + body)
    assert bench.recorded_traffic("box-2d3r-f64-T2-valu") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_paper_cases_table_is_table3():
    # the six cases of the paper's Table 3: (pattern, fusion depth, type)
    got = [(c[1], c[2], c[3], c[4], c[5]) for c in bench.PAPER_CASES]
    assert got == [("box", 2, 1, 3, "f64"), ("box", 2, 3, 1, "f64"), ("box", 2, 1, 7, "f32"),
                   ("box", 2, 7, 1, "f32"), ("box", 3, 1, 3, "f64"), ("box", 3, 1, 7, "f32")]
    # the A100 rates the bench quotes as context are the table's
    cases = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))["table3"]["cases"]
    for c, g in zip(bench.PAPER_CASES, cases):
        assert (c[1], c[2], c[3], c[4]) == (g["shape"], g["d"], g["r"], g["t"])
        assert c[5] == {"double": "f64", "float": "f32"}[g["dtype"]]
        assert c[6] == (g["cu"]["gst"], g["tc"]["gst"])


def _synthetic_sections():
    variants = {}
    for shape in ("box", "star"):
        for dt in ("f64", "f32"):
            for T in (1, 2, 4):
                for path in ("valu", "mfma"):
                    variants[f"{shape}-2d3r-{dt}-T{T}-{path}"] = {
                        "gst": 1234.5678, "ms_per_sweep": 12.3456, "path": path,
                        "roofline": {"bound": "alu", "achieved": 33.3333, "peak": 78.6,
                                     "unit": "TFLOP/s", "frac": 0.4241}}
    mcheck = {"agree": 36, "total": 36, "cases": [{"case": "x"}] * 36}
    precision = {"reference": {"gst": 500.0}}
    for k in ("bf16-mfma-T4", "f16-mfma-T4", "bf16x3-mfma-T4", "bf16-mfma-T2", "bf16-valu-T2",
              "f16-valu-T2", "f32-valu-T2", "f32-mfma-T4"):
        precision[k] = {"gst": 2434.123456, "err_every_100": [1e-3] * 10,
                        "oracle_e2e_1000": 0.0595123456, "oracle_arith_1000": 0.0123456789}
    lat = {"p50_ms": 5.0345, "p99_ms": 106.0871, "gst": 138.0603}
    serving = {"served": lat, "fifo": lat, "served_capacity": {"gst": 231.04}, "fifo_capacity": {"gst": 175.9}}
    cases = {str(i): {"valu": {"gst": 799.43}, "mfma": {"gst": 485.59}, "predicted": "valu",
                      "measured": "valu"} for i in range(1, 7)}
    return variants, mcheck, precision, serving, cases


def test_json_line_is_small_and_complete():
    import argparse
    variants, mcheck, precision, serving, cases = _synthetic_sections()
    args = argparse.Namespace(steps=20, warmup=5, n=8192, time_steps=100)
    head_name = "box-2d3r-f64-T2-valu"
    hv = next(v for v in bench.headline_variants(8192, 100) if v["name"] == head_name)
    roof = dict(variants[head_name]["roofline"], traffic=1.133e9)
    cpu = {"value": 0.1153456, "unit": "GStencil/s", "cores": 16, "kind": "oracle",
           "sample": "Box-2D3R f64 8192x8192, 16 time steps (of 100), zero Dirichlet halo",
           "cpu_model": "AMD EPYC 9575F 64-Core Processor", "nproc": 256, "affinity": 16}
    clocks = {"sclk_mhz": 2400, "mclk_mhz": 1900, "fclk_mhz": 2000, "socclk_mhz": 1200}
    sparse = {f"box-2d{r}r-bf16-T{T}-{n}": {"mfma": {"gst": 1234.567}, "mfma_sparse": {"gst": 1534.567},
                                            "model_speedup": 1.25} for r, T, n in ((1, 7, 10240), (2, 3, 16384),
                                                                                   (3, 2, 8192), (3, 2, 8193))}
    seq = {f"{sh}-2d3r-{dt}-T{T}-8192": {"mfma": 123.456, "mfma_seq": 111.111} for sh in ("box", "star")
           for dt in ("f64", "f32") for T in (2, 4)}
    grid = {"agree": 32, "total": 32}
    summ = bench.summaries(variants, mcheck, precision, serving, cases, sparse, grid, seq)
    s = bench.compact_line(args, head_name, variants[head_name], hv, roof, cpu, clocks, summ)
    assert len(s.encode()) <= 4096, len(s)
    line = json.loads(s)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "clocks"):
        assert k in line, k
    assert line["dtype"] == "f64" and line["n_gpus"] == 1 and line["steps"] == 20
    assert "workload" in line["config"] and "model" not in line["config"]
    assert set(line["roofline"]) >= {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert set(line["cpu_baseline"]) >= {"value", "unit", "cores", "kind", "sample", "cpu_model", "nproc"}
    assert line["summary"]["model_check"] == "36/36"
    assert len(line["summary"]["precision"]["bf16-mfma-T4"]) == 3
    assert line["summary"]["serving"]["served"] == [5.03, 106.09, 138.1]


def test_case_names_and_the_measured_ceiling_column():
    """Variant names parse into (shape, d, r, dtype, T); the model's second
    column takes per-dtype ceilings and changes the verdict only through them:
    with the datasheet ceilings it equals the first column, and with a vector
    unit far slower than the matrix unit the MFMA path wins."""
    import paper_2603_00477_amd as stl
    assert bench.parse_case("box-2d3r-f64-T2") == ("box", 2, 3, "f64", 2)
    assert bench.parse_case("star-3d2r-f32-T3-valu") == ("star", 3, 2, "f32", 3)
    assert bench.parse_case("no such case") is None
    dt = "f64"
    datasheet = stl.hw_default(dt) if hasattr(stl, "hw_default") else None
    if datasheet is not None:
        hw = {"per_dtype": {dt: datasheet}}
        m = stl.model_predict("box", 2, 3, 2, dt)
        assert bench.predicted_with(stl, hw, "box-2d3r-f64-T2") == {-1: "valu", 0: "tie", 1: "mfma"}[m["winner"]]
    slow_valu = {"per_dtype": {dt: dict(BB=8e12, PP_valu=1e11, PP_mfma=78.6e12, PP_mfma_sparse=157.2e12)}}
    assert bench.predicted_with(stl, slow_valu, "box-2d3r-f64-T1") == "mfma"
    assert bench.predicted_with(stl, None, "box-2d3r-f64-T1") is None
