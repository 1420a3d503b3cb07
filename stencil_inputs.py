"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module only draws random numbers and lays them out; it performs none of
the stencil arithmetic (no offsets, no weighted sums, no composition).  Both
the CPU oracle (``oracle/``) and the GPU library's tests and benchmark take
their grids and weight vectors from here, so that the two sides see identical
bytes.

Conventions
-----------
* Random numbers come from ``numpy.random.Generator(PCG64(seed))``.
* Grids are generated in float64, dense, C-contiguous, slowest axis first.
* Weight vectors have length K (the caller supplies K for its shape), are drawn
  uniform on [0, 1) and normalised so that they sum to one, in float64.
* Seeds follow the workload numbering: data ``1000*c + v``, weights
  ``1000*c + 500 + v`` (workload c = 1..5, variant index v).
* ``round_to`` rounds a float64 array to a storage type with round-to-nearest-
  even and returns both the rounded float64 values and the storage tensor
  bytes (as a torch CPU tensor) for upload.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng",
    "data_seed",
    "weight_seed",
    "uniform_grid",
    "smooth_grid",
    "normalised_weights",
    "dyadic_grid",
    "dyadic_weights",
    "round_to",
    "served_trace",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def data_seed(workload: int, variant: int = 0) -> int:
    return 1000 * int(workload) + int(variant)


def weight_seed(workload: int, variant: int = 0) -> int:
    return 1000 * int(workload) + 500 + int(variant)


def uniform_grid(dims, seed: int) -> np.ndarray:
    """Grid of shape ``dims`` with values uniform on [0, 1), float64."""
    g = rng(seed)
    return g.random(tuple(int(n) for n in dims), dtype=np.float64)


def smooth_grid(dims, seed: int, noise: float = 1e-3) -> np.ndarray:
    """sin(2*pi*x) * sin(2*pi*y) + noise * U[0,1) on a 2D grid.

    x = j / n1 runs along the fastest axis, y = i / n0 along the slowest.
    """
    n0, n1 = (int(n) for n in dims)
    y = np.arange(n0, dtype=np.float64)[:, None] / n0
    x = np.arange(n1, dtype=np.float64)[None, :] / n1
    base = np.sin(2.0 * math.pi * x) * np.sin(2.0 * math.pi * y)
    return base + noise * rng(seed).random((n0, n1), dtype=np.float64)


def normalised_weights(K: int, seed: int) -> np.ndarray:
    """K weights drawn uniform on [0, 1) and divided by their sum (float64)."""
    w = rng(seed).random(int(K), dtype=np.float64)
    return w / w.sum()


def dyadic_grid(dims, seed: int, bits: int = 8) -> np.ndarray:
    """Grid of small dyadic rationals k / 2**bits, k uniform in [0, 2**bits).

    Sums of products of such values with dyadic weights are exact in float64
    while the denominators stay below 2**53.
    """
    g = rng(seed)
    k = g.integers(0, 1 << bits, size=tuple(int(n) for n in dims))
    return k.astype(np.float64) / float(1 << bits)


def dyadic_weights(K: int, seed: int, bits: int = 6) -> np.ndarray:
    """K dyadic weights k / 2**bits with k uniform in [1, 2**bits)."""
    g = rng(seed)
    k = g.integers(1, 1 << bits, size=int(K))
    return k.astype(np.float64) / float(1 << bits)


_STORAGE = {
    "f64": "float64",
    "f32": "float32",
    "bf16": "bfloat16",
    "f16": "float16",
    # compensated mode stores float32
    "bf16x3": "float32",
}


def round_to(a: np.ndarray, dtype: str):
    """Round float64 ``a`` to storage type ``dtype`` (RNE).

    Returns ``(values_f64, tensor)`` where ``values_f64`` holds the rounded
    values widened back to float64 and ``tensor`` is a contiguous torch CPU
    tensor of the storage type holding the same values.
    """
    import torch

    tdt = getattr(torch, _STORAGE[dtype])
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(tdt).contiguous()
    return t.to(torch.float64).numpy(), t


def served_trace(n_jobs: int, seed: int = 5000, rate_per_s: float = 1000.0,
                 side2d=(256, 8192), side3d=(64, 512), steps=(1, 64),
                 radii=(1, 2, 3)):
    """Seeded stream of stencil jobs with Poisson arrivals.

    Each job is a dict with arrival time (seconds), shape ('star'|'box'),
    d (2|3), r, dims (square/cubic side drawn log-uniform in the given range),
    steps (uniform integer), boundary ('dirichlet'|'periodic') and the seeds
    for its data and weights.
    """
    g = rng(seed)
    t = 0.0
    jobs = []
    for i in range(int(n_jobs)):
        t += g.exponential(1.0 / rate_per_s)
        shape = "star" if g.random() < 0.5 else "box"
        d = 2 if g.random() < 0.5 else 3
        r = int(radii[int(g.integers(0, len(radii)))])
        lo, hi = side2d if d == 2 else side3d
        side = int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))
        st = int(g.integers(steps[0], steps[1] + 1))
        boundary = "dirichlet" if g.random() < 0.5 else "periodic"
        jobs.append(dict(id=i, arrival=t, shape=shape, d=d, r=r,
                         dims=(side,) * d, steps=st, boundary=boundary,
                         data_seed=seed * 10 + 2 * i, weight_seed=seed * 10 + 2 * i + 1))
    return jobs
