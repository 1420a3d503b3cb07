"""Parity at the benchmark's own sizes, in the launch configurations the
benchmark times.

Each test runs the same plans as the benchmark (same grid, dtype, boundary,
fusion depth T, path and number of time steps) and compares sampled windows
of the output with the FP64 oracle, evaluated on the window's dependency cone
only (oracle.core.run_window, bit-identical to the full-grid oracle).  The
windows sit on corners and edges (boundary rule, periodic wrap), on the
Dirichlet band that kernel-fused MFMA passes recompute (width r (T - 1)), on
tile seams of both kernel families (multiples of 64 / 128 / 1024 columns and
the row midpoint) and in the interior.

On top of the windows, every variant's whole output is compared with the
float64 VALU result of the same workload, itself checked on the windows.

Tolerances (relative max-norm, reading of the paper's precision protocol):
float64 <= 1e-12; float32 <= 1e-5 against the oracle on the float64 data.
16-bit and compensated modes: absolute error against the oracle on the
storage-rounded data (arithmetic error) within the worst-case bound
    passes * (u_store + u_w + K_T 2^-24) * max|u0|
for a non-expansive operator (weights >= 0, summing to 1)."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import stencil_inputs as si
from gpu_util import lowp_bound
from oracle import core as ocore
from oracle import model as omodel

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def stl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_00477_amd as stl
    stl.lib()
    return stl


def windows2d(n, s=16):
    """(lo, hi) boxes of side s: corners, edges, the fix-up band edge, tile
    seams and the interior of an n x n grid."""
    m = n // 2
    starts = [(0, 0), (n - s, n - s), (0, m - s // 2), (m - s // 2, 0), (n - s, 1017),
              (2, 3000), (m - s // 2, 1024 - s // 2), (m + 61, n - 128 - s // 2),
              (4099, 6135)]
    return [((a, b), (a + s, b + s)) for a, b in starts]


def windows3d(n, s=8):
    m = n // 2
    starts = [(0, 0, 0), (n - s, n - s, n - s), (m - s // 2, 60, 252), (301, n - s, 0),
              (17, 131, 443)]
    return [((a, b, c), (a + s, b + s, c + s)) for a, b, c in starts]


def _slice(lo, hi):
    return tuple(slice(a, b) for a, b in zip(lo, hi))


def _run(stl, shape, d, r, w, dims, T, dt, path, boundary, x, steps):
    import torch
    p = stl.Plan(shape, d, r, w, dims, T=T, dtype=dt, path=path, boundary=boundary)
    info = p.info()
    assert info["path_name"] == path and info["T"] == T
    y = torch.empty_like(x)
    p.run(x, y, steps)
    torch.cuda.synchronize()
    p.close()
    return y


def _check_variants(stl, shape, d, r, K, dims, steps, boundary, Ts, u0, w, wins):
    """Run every (dtype, T, path) variant, compare windows with the oracle and
    whole outputs with the float64 VALU result."""
    import torch
    refs = [ocore.run_window(shape, d, r, w, u0, steps, lo, hi, boundary) for lo, hi in wins]
    scale = max(float(np.max(np.abs(rf))) for rf in refs)
    base = None
    report = []
    for dt in ("f64", "f32"):
        x = si.round_to(u0, dt)[1].to("cuda")
        for T in Ts:
            for path in ("valu", "mfma"):
                print(f"[fullsize] {shape}-{d}d{r}r {dt} T={T} {path} {dims} {steps} steps",
                      flush=True)
                y = _run(stl, shape, d, r, w, dims, T, dt, path, boundary, x, steps)
                werr = max(float(np.max(np.abs(y[_slice(lo, hi)].to(torch.float64).cpu().numpy() - rf)))
                           for (lo, hi), rf in zip(wins, refs)) / scale
                yd = y.to(torch.float64)
                if base is None:
                    assert dt == "f64" and path == "valu"
                    assert werr <= TOL["f64"], (dt, T, path, werr)
                    base = yd
                    ferr = 0.0
                else:
                    ferr = float((yd - base).abs().max() / base.abs().max())
                report.append((dt, T, path, werr, ferr))
                assert werr <= TOL[dt], (dt, T, path, "window", werr)
                assert ferr <= TOL[dt], (dt, T, path, "whole grid vs f64 VALU", ferr)
                del y, yd
        del x
        torch.cuda.empty_cache()
    for row in report:
        print("[fullsize] %s T=%d %s: window err %.2e, whole-grid err %.2e" % row, flush=True)


@pytest.mark.parametrize("shape,r,K", [("box", 3, 49), ("star", 3, 13)])
def test_workload_8192_dirichlet_100_steps(stl, shape, r, K):
    """Box-2D3R / Star-2D3R, 8192^2, zero Dirichlet halo, 100 steps, float64
    and float32, T in {1, 2, 4}, VALU and MFMA: the benchmark's sweeps."""
    n = 8192
    u0 = si.uniform_grid((n, n), seed=si.data_seed(2, 0))
    w = si.normalised_weights(K, seed=si.weight_seed(2, 0 if shape == "box" else 1))
    _check_variants(stl, shape, 2, r, K, (n, n), 100, "dirichlet", (1, 2, 4), u0, w, windows2d(n))


@pytest.mark.parametrize("shape,r,K,vi", [("star", 2, 13, 0), ("box", 1, 27, 1)])
def test_workload_512cube_periodic_50_steps(stl, shape, r, K, vi):
    """Star-3D2R / Box-3D1R, 512^3, periodic, 50 steps, float64 and float32,
    T in {1, 2, 3} (T = 3 ends with a two-step remainder pass), VALU and
    MFMA: the benchmark's sweeps."""
    n = 512
    u0 = si.uniform_grid((n, n, n), seed=si.data_seed(3, 0))
    w = si.normalised_weights(K, seed=si.weight_seed(3, vi))
    _check_variants(stl, shape, 3, r, K, (n, n, n), 50, "periodic", (1, 2, 3), u0, w, windows3d(n))


def _golden16384():
    with open(os.path.join(HERE, "golden", "precision_windows_16384.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("dt", ["bf16", "f16", "bf16x3"])
def test_workload_16384_precision_1000_steps(stl, dt):
    """Box-2D2R, 16384^2, periodic, smooth data, T = 4 MFMA in bf16 / f16
    with float32 accumulation and the compensated bf16x3 mode: 1000 steps in
    ten runs of 100 as the benchmark does.  Windows after 100 steps against
    the live oracle, after 1000 steps against stored oracle values; both the
    arithmetic error (oracle on the storage-rounded data) within the stated
    bound and the end-to-end error (oracle on the float64 data) reported."""
    import torch
    n, T, steps = 16384, 4, 1000
    g = _golden16384()
    u0 = si.smooth_grid((n, n), seed=si.data_seed(4, 0))
    w = si.normalised_weights(25, seed=si.weight_seed(4, 0))
    assert np.array_equal(np.asarray(g["weights"]), w)
    import hashlib
    assert hashlib.sha1(u0.tobytes()).hexdigest() == g["u0_sha1"]
    store = {"bf16": "bf16", "f16": "f16", "bf16x3": "f32"}[dt]
    u0r, t = si.round_to(u0, store)
    wins = windows2d(n)[:5]
    ref100_r = [ocore.run_window("box", 2, 2, w, u0r, 100, lo, hi, "periodic") for lo, hi in wins]
    ref100 = [ocore.run_window("box", 2, 2, w, u0, 100, lo, hi, "periodic") for lo, hi in wins]
    p = stl.Plan("box", 2, 2, w, (n, n), T=T, dtype=dt, path="mfma", boundary="periodic")
    assert p.info()["path_name"] == "mfma"
    x = t.to("cuda")
    y = torch.empty_like(x)
    print(f"[fullsize] box-2d2r {dt} T={T} mfma {n}^2 periodic, 10 x 100 steps", flush=True)
    snaps = {}
    for k in range(10):
        p.run(x, y, 100)
        x, y = y, x
        if k in (0, 9):
            snaps[(k + 1) * 100] = x.to(torch.float64)
    torch.cuda.synchronize()
    umax = float(np.max(np.abs(u0r)))
    K_T = omodel.K_fused("box", 2, 2, T)
    lo, hi = g["lo"], g["hi"]
    gw = np.asarray(g["windows"][store]["values"])
    gw_e2e = np.asarray(g["windows"]["f64"]["values"])
    res = {}
    for st, arith_refs, e2e_refs, boxes in ((100, ref100_r, ref100, wins),
                                            (1000, [gw], [gw_e2e], [(lo, hi)])):
        got = [snaps[st][_slice(a, b)].cpu().numpy() for a, b in boxes]
        arith = max(float(np.max(np.abs(gg - rf))) for gg, rf in zip(got, arith_refs))
        e2e = max(float(np.max(np.abs(gg - rf))) for gg, rf in zip(got, e2e_refs))
        bound = lowp_bound(dt, K_T, st // T, umax)
        res[st] = (arith, e2e, bound)
        print(f"[fullsize] {dt} after {st} steps: arithmetic error {arith:.3e} (bound {bound:.3e}), "
              f"end-to-end error {e2e:.3e}", flush=True)
        assert arith <= bound, (dt, st, arith, bound)
    p.close()


def test_workload_16384_f64_reference_1000_steps(stl):
    """The float64 VALU sweep the benchmark uses as the whole-grid reference
    of the precision workload (T = 2, 1000 steps in ten runs of 100) equals
    the FP64 oracle on the stored window after 1000 steps and on live windows
    after 100 steps (relative 1e-12)."""
    import torch
    n = 16384
    g = _golden16384()
    u0 = si.smooth_grid((n, n), seed=si.data_seed(4, 0))
    w = si.normalised_weights(25, seed=si.weight_seed(4, 0))
    wins = windows2d(n)[:5]
    ref100 = [ocore.run_window("box", 2, 2, w, u0, 100, lo, hi, "periodic") for lo, hi in wins]
    p = stl.Plan("box", 2, 2, w, (n, n), T=2, dtype="f64", path="valu", boundary="periodic")
    x = torch.from_numpy(u0).to("cuda")
    y = torch.empty_like(x)
    print(f"[fullsize] box-2d2r f64 T=2 valu {n}^2 periodic, 10 x 100 steps", flush=True)
    for k in range(10):
        p.run(x, y, 100)
        x, y = y, x
        if k == 0:
            got = [x[_slice(a, b)].cpu().numpy() for a, b in wins]
            scale = max(float(np.max(np.abs(rf))) for rf in ref100)
            err = max(float(np.max(np.abs(gg - rf))) for gg, rf in zip(got, ref100)) / scale
            assert err <= 1e-12, err
    torch.cuda.synchronize()
    lo, hi = g["lo"], g["hi"]
    gw = np.asarray(g["windows"]["f64"]["values"])
    err = float(np.max(np.abs(x[_slice(lo, hi)].cpu().numpy() - gw)) / np.max(np.abs(gw)))
    print(f"[fullsize] f64 reference after 1000 steps: {err:.2e}", flush=True)
    assert err <= 1e-12, err
    p.close()
