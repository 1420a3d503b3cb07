"""Helpers shared by the GPU tests: seeded inputs onto the device, oracle
references, error norms.  Inputs come from stencil_inputs; expected values
come only from the oracle."""
from __future__ import annotations

import numpy as np

import stencil_inputs as si
from oracle import core as ocore
from oracle import model as omodel

DT = {"f64": "f64", "f32": "f32", "bf16": "bf16", "f16": "f16", "bf16x3": "bf16x3"}

# Unit roundoff of the storage types (2^-p for a p-bit significand: bf16 8,
# f16 11, float32 24; the compensated mode stores float32).
U_STORE = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11, "bf16x3": 2.0 ** -24, "f32": 2.0 ** -24}
# Relative error per product from the operands of an MFMA pass: the composite
# weights rounded once to bf16 / f16 (unit roundoff), or, for the compensated
# hi/lo split, three terms of up to 2^-16 each: the weight-split residual
# (w - w_hi - w_lo), the data-split residual (x - x_hi - x_lo) and the
# dropped w_lo * x_lo product.
U_W = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11, "bf16x3": 3 * 2.0 ** -16}


def lowp_bound(dt, K_T, passes, umax):
    """Worst-case absolute error of `passes` MFMA passes in a 16-bit or
    compensated mode, for a non-expansive operator (weights >= 0 summing to
    1, so errors of earlier passes are not amplified): per pass the stored
    result rounds once (u_store), every product carries at most u_w, and
    float32 accumulation of K_T terms adds at most K_T 2^-24, all relative to
    max|u| <= max|u0| (maximum principle)."""
    return passes * (U_STORE[dt] + U_W[dt] + K_T * 2.0 ** -24) * umax


def rel_inf(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def case_inputs(shape, d, r, dims, dtype, seed):
    """(u0 float64, u0 rounded to dtype as float64, torch storage tensor, weights f64)."""
    K = omodel.K_points(shape, d, r)
    w = si.normalised_weights(K, seed=seed + 500)
    u0 = si.uniform_grid(dims, seed=seed)
    u0r, t = si.round_to(u0, dtype)
    return u0, u0r, t, w


def run_gpu(plan, t_in, steps):
    import torch
    x = t_in.to("cuda")
    y = torch.empty_like(x)
    plan.run(x, y, steps)
    torch.cuda.synchronize()
    return y.to(torch.float64).cpu().numpy()


def oracle(shape, d, r, w, u0, steps, boundary, halo=0.0):
    return ocore.run(shape, d, r, w, u0, steps, boundary, halo)
