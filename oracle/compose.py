"""Composite kernel of kernel fusion (test infrastructure only).

Fusing t explicit steps into one monolithic step (paper, Sec. "Handling
Stencils with Small Radius" and the fusion-redundancy example) replaces the
K-point kernel of radius r by a kernel of radius t*r.  With the step
u'[x] = sum_o w[o] u[x+o], two steps give u''[x] = sum_{o,p} w[o] w[p]
u[x+o+p], so the composite weight of displacement q is the sum of the products
of t weights whose displacements add up to q: the t-fold full convolution of
the weight pattern with itself.  For a periodic grid (or away from a
Dirichlet boundary by at least r*(t-1)) one application of the composite
equals t steps.
"""
from __future__ import annotations

import numpy as np

from . import core


def dense_kernel(shape, d: int, r: int, weights) -> np.ndarray:
    """Single-step weights as a dense (2r+1)^d array indexed by offset + r."""
    offs = core.offsets(shape, d, r)
    W = np.zeros((2 * r + 1,) * d, dtype=np.float64)
    for k, o in enumerate(offs):
        W[tuple(int(c) + r for c in o)] += float(weights[k])
    return W


def composite(shape, d: int, r: int, weights, t: int) -> np.ndarray:
    """t-fold composite kernel, dense (2rt+1)^d float64, indexed by offset + rt."""
    base = dense_kernel(shape, d, r, weights)
    W = base.copy()
    for s in range(1, int(t)):
        R_old = r * s
        R_new = r * (s + 1)
        new = np.zeros((2 * R_new + 1,) * d, dtype=np.float64)
        for idx in np.ndindex(*base.shape):
            wv = base[idx]
            if wv == 0.0:
                continue
            # displacement o = idx - r shifts the old kernel (indexed by q + R_old)
            sl = tuple(slice(i, i + 2 * R_old + 1) for i in idx)
            new[sl] += wv * W
        W = new
    return W


def support_size(shape, d: int, r: int, t: int) -> int:
    """Number of displacements the composite couples (generic positive weights)."""
    K = core.num_points(shape, d, r)
    w = np.linspace(1.0, 2.0, K)
    return int(np.count_nonzero(composite(shape, d, r, w, t)))


def apply_composite_periodic(Wc: np.ndarray, u: np.ndarray) -> np.ndarray:
    """One application of a dense composite kernel on a periodic grid (float64),
    summing displacements in row-major order."""
    R = (Wc.shape[0] - 1) // 2
    out = np.zeros_like(u, dtype=np.float64)
    for idx in np.ndindex(*Wc.shape):
        wv = Wc[idx]
        if wv == 0.0:
            continue
        disp = tuple(i - R for i in idx)
        out = out + wv * np.roll(u, shift=tuple(-c for c in disp), axis=tuple(range(u.ndim)))
    return out
