"""ctypes front end of the C oracle (``stencil_oracle.c``).

Test infrastructure only.  Shapes, boundaries and offsets follow the paper's
problem statement (Introduction; Sec. "Original Stencil Problem"): a weighted
sum over the K points of a box or star pattern of radius r in d dimensions,
applied as explicit out-of-place steps.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

SHAPES = {"star": 0, "box": 1}
BOUNDARIES = {"dirichlet": 0, "periodic": 1}

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_offsets.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_int)]
        L.oracle_offsets.restype = ctypes.c_int
        L.oracle_run_window.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, i64p,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp,
                                        i64p, i64p, dp, ctypes.c_int]
        L.oracle_run_window.restype = ctypes.c_int
        L.oracle_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, i64p,
                                 ctypes.c_int, ctypes.c_double, ctypes.c_int64, dp, dp,
                                 ctypes.c_int]
        L.oracle_run.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _shape(s):
    return SHAPES[s] if isinstance(s, str) else int(s)


def _bnd(b):
    return BOUNDARIES[b] if isinstance(b, str) else int(b)


def num_points(shape, d: int, r: int) -> int:
    """K of the pattern: (2r+1)^d for box, 2dr+1 for star."""
    return int(lib().oracle_offsets(_shape(shape), int(d), int(r), None))


def offsets(shape, d: int, r: int) -> np.ndarray:
    """(K, d) int array of offsets in canonical order."""
    K = num_points(shape, d, r)
    buf = (ctypes.c_int * (K * d))()
    lib().oracle_offsets(_shape(shape), int(d), int(r), buf)
    return np.frombuffer(buf, dtype=np.int32).reshape(K, d).astype(np.int64)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def run(shape, d: int, r: int, weights, u0, steps: int, boundary="dirichlet",
        halo: float = 0.0, threads: int = 0) -> np.ndarray:
    """step^steps(u0) over the whole grid, float64."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    assert u0.ndim == d and w.size == num_points(shape, d, r)
    dims = np.array(u0.shape, dtype=np.int64)
    out = np.empty_like(u0)
    rc = lib().oracle_run(_shape(shape), d, r, _dp(w), _ip(dims), _bnd(boundary), float(halo),
                          int(steps), _dp(u0), _dp(out), int(threads))
    if rc != 0:
        raise ValueError(f"oracle_run failed with code {rc}")
    return out


def run_window(shape, d: int, r: int, weights, u0, steps: int, lo, hi,
               boundary="dirichlet", halo: float = 0.0, threads: int = 0) -> np.ndarray:
    """step^steps(u0) restricted to the box [lo, hi), float64 (bit-identical
    to the corresponding slice of ``run``)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    assert u0.ndim == d and w.size == num_points(shape, d, r)
    dims = np.array(u0.shape, dtype=np.int64)
    lo = np.array(lo, dtype=np.int64)
    hi = np.array(hi, dtype=np.int64)
    out = np.empty(tuple(int(x) for x in (hi - lo)), dtype=np.float64)
    rc = lib().oracle_run_window(_shape(shape), d, r, _dp(w), _ip(dims), _bnd(boundary),
                                 float(halo), int(steps), _dp(u0), _ip(lo), _ip(hi), _dp(out),
                                 int(threads))
    if rc != 0:
        raise ValueError(f"oracle_run_window failed with code {rc}")
    return out


def max_threads() -> int:
    return int(lib().oracle_max_threads())
