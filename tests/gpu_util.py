"""Helpers shared by the GPU tests: seeded inputs onto the device, oracle
references, error norms.  Inputs come from stencil_inputs; expected values
come only from the oracle."""
from __future__ import annotations

import numpy as np

import stencil_inputs as si
from oracle import core as ocore
from oracle import model as omodel

DT = {"f64": "f64", "f32": "f32", "bf16": "bf16", "f16": "f16", "bf16x3": "bf16x3"}


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
