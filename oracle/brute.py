"""Brute-force step operator for tiny grids (pure Python, exact rationals).

Test infrastructure only.  Written independently of the C oracle's offset
loop: it enumerates every (output point, input point) pair of the grid and
decides from the displacement alone whether the pair is coupled, following
the paper's description of the two patterns (Introduction): a box couples
every displacement whose largest coordinate magnitude is at most r; a star
couples the displacements that lie on one coordinate axis within distance r.

The weight of a coupled displacement is looked up by position in the weight
vector (box: row-major over displacements, last axis fastest; star: centre,
then per axis the displacements -r..-1, +1..+r).  Out-of-grid neighbours of
a Dirichlet problem contribute weight * h to a constant term; for a periodic
problem the displacement is taken modulo the grid, and all displacements that
alias to the same input point are summed (relevant when n < 2r + 1).

``operator`` returns (A, b) with u' = A u + b over Fractions; ``apply`` runs
N steps exactly.
"""
from __future__ import annotations

import itertools
from fractions import Fraction


def _weight_index(shape: str, d: int, r: int, disp):
    """Position of displacement ``disp`` in the weight vector, or None."""
    if shape == "box":
        if max(abs(c) for c in disp) > r:
            return None
        idx = 0
        for c in disp:
            idx = idx * (2 * r + 1) + (c + r)
        return idx
    nz = [i for i, c in enumerate(disp) if c != 0]
    if not nz:
        return 0
    if len(nz) > 1:
        return None
    ax = nz[0]
    c = disp[ax]
    if abs(c) > r:
        return None
    within = c + r if c < 0 else c + r - 1
    return 1 + ax * 2 * r + within


def _points(dims):
    return list(itertools.product(*[range(n) for n in dims]))


def operator(shape: str, dims, r: int, weights, boundary: str = "dirichlet", halo=0):
    """Affine step operator on a grid of shape ``dims`` as (A, b), where A is a
    dict-of-dicts {out_lin: {in_lin: Fraction}} and b a list of Fractions."""
    d = len(dims)
    w = [Fraction(x) for x in weights]
    h = Fraction(halo)
    pts = _points(dims)
    lin = {p: i for i, p in enumerate(pts)}
    A = {i: {} for i in range(len(pts))}
    b = [Fraction(0)] * len(pts)
    if boundary == "dirichlet":
        # every displacement within the pattern's bounding box
        rng = range(-r, r + 1)
        for p in pts:
            i = lin[p]
            for disp in itertools.product(rng, repeat=d):
                k = _weight_index(shape, d, r, disp)
                if k is None:
                    continue
                q = tuple(pc + dc for pc, dc in zip(p, disp))
                if all(0 <= qc < n for qc, n in zip(q, dims)):
                    j = lin[q]
                    A[i][j] = A[i].get(j, Fraction(0)) + w[k]
                else:
                    b[i] += w[k] * h
    else:
        for p in pts:
            i = lin[p]
            for disp in itertools.product(range(-r, r + 1), repeat=d):
                k = _weight_index(shape, d, r, disp)
                if k is None:
                    continue
                q = tuple((pc + dc) % n for pc, dc, n in zip(p, disp, dims))
                j = lin[q]
                A[i][j] = A[i].get(j, Fraction(0)) + w[k]
    return A, b


def apply(shape: str, u0, r: int, weights, steps: int, boundary: str = "dirichlet", halo=0):
    """N exact steps on a nested-list / numpy grid; returns a flat list of
    Fractions in row-major order."""
    import numpy as np

    arr = np.asarray(u0)
    dims = arr.shape
    A, b = operator(shape, dims, r, weights, boundary, halo)
    u = [Fraction(float(x)) for x in arr.reshape(-1)]
    for _ in range(int(steps)):
        u = [sum((a * u[j] for j, a in A[i].items()), Fraction(0)) + b[i] for i in range(len(u))]
    return u
