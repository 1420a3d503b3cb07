"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Step operator (paper, Introduction; Sec. "Original Stencil Problem"):
  * exact-rational brute force on tiny grids (independent operator builder),
  * scipy.ndimage.correlate for one step,
  * FFT eigenvalues for periodic N steps, and the closed form for the
    sin(2 pi x) sin(2 pi y) modes,
  * invariants: constants, linear fields, quadratic growth, linearity,
    maximum principle,
  * window evaluation bit-identical to the full grid.
Composite kernel of kernel fusion (Sec. "Handling Stencils with Small Radius"):
  * one composite application equals t steps (periodic, exact), support sizes.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

import stencil_inputs as si
from oracle import brute, compose, core, model

CASES_TINY = [
    ("star", (7, 9), 1), ("star", (6, 8), 2), ("box", (7, 9), 1), ("box", (6, 7), 2),
    ("star", (4, 5, 6), 1), ("box", (4, 5, 6), 1), ("star", (5, 4, 6), 2),
]


@pytest.mark.parametrize("shape,dims,r", CASES_TINY)
@pytest.mark.parametrize("boundary,halo", [("dirichlet", 0.0), ("dirichlet", 0.5), ("periodic", 0.0)])
def test_brute_force_exact(shape, dims, r, boundary, halo):
    d = len(dims)
    K = model.K_points(shape, d, r)
    w = si.dyadic_weights(K, seed=11 + r)
    u0 = si.dyadic_grid(dims, seed=7 + d)
    steps = 2 if d == 3 else 3
    exact = brute.apply(shape, u0, r, w, steps, boundary, halo)
    got = core.run(shape, d, r, w, u0, steps, boundary, halo)
    # dyadic data and weights: every FP64 operation is exact here
    assert [float(x) for x in exact] == got.reshape(-1).tolist()


def test_brute_force_periodic_aliasing():
    """Grid smaller than the pattern: aliased displacements are summed."""
    w = si.dyadic_weights(25, seed=3)
    u0 = si.dyadic_grid((3, 4), seed=4)
    exact = brute.apply("box", u0, 2, w, 2, "periodic")
    got = core.run("box", 2, 2, w, u0, 2, "periodic")
    assert [float(x) for x in exact] == got.reshape(-1).tolist()


def test_brute_force_generic_weights_close():
    """Non-dyadic weights: FP64 within a few ulps of the exact rational."""
    w = si.normalised_weights(9, seed=5)
    u0 = si.uniform_grid((6, 7), seed=6)
    exact = brute.apply("box", u0, 1, w, 4, "dirichlet")
    got = core.run("box", 2, 1, w, u0, 4, "dirichlet").reshape(-1)
    err = max(abs(float(e) - g) for e, g in zip(exact, got))
    assert err < 1e-14


@pytest.mark.parametrize("shape,d,r", [("star", 2, 1), ("box", 2, 3), ("star", 2, 3),
                                       ("box", 3, 1), ("star", 3, 2)])
@pytest.mark.parametrize("boundary", ["dirichlet", "periodic"])
def test_scipy_correlate_one_step(shape, d, r, boundary):
    dims = (33, 41) if d == 2 else (13, 11, 17)
    K = model.K_points(shape, d, r)
    w = si.normalised_weights(K, seed=21)
    u0 = si.uniform_grid(dims, seed=22)
    dense = np.zeros((2 * r + 1,) * d)
    for k, o in enumerate(core.offsets(shape, d, r)):
        dense[tuple(o + r)] = w[k]
    if boundary == "dirichlet":
        ref = ndi.correlate(u0, dense, mode="constant", cval=0.25)
        got = core.run(shape, d, r, w, u0, 1, boundary, 0.25)
    else:
        ref = ndi.correlate(u0, dense, mode="wrap")
        got = core.run(shape, d, r, w, u0, 1, boundary)
    assert np.max(np.abs(ref - got)) < 1e-14


def _fft_steps(shape, d, r, w, u0, steps):
    offs = core.offsets(shape, d, r)
    lam = np.zeros(u0.shape, dtype=np.complex128)
    grids = np.meshgrid(*[np.arange(n) for n in u0.shape], indexing="ij")
    for k, o in enumerate(offs):
        phase = sum(2j * np.pi * grids[i] * o[i] / u0.shape[i] for i in range(d))
        lam += w[k] * np.exp(phase)
    return np.real(np.fft.ifftn(np.fft.fftn(u0) * lam ** steps))


@pytest.mark.parametrize("shape,d,r,steps", [("box", 2, 2, 20), ("star", 2, 3, 15),
                                             ("box", 3, 1, 6), ("star", 3, 2, 5)])
def test_fft_periodic(shape, d, r, steps):
    dims = (24, 20) if d == 2 else (10, 12, 9)
    w = si.normalised_weights(model.K_points(shape, d, r), seed=31)
    u0 = si.uniform_grid(dims, seed=32)
    ref = _fft_steps(shape, d, r, w, u0, steps)
    got = core.run(shape, d, r, w, u0, steps, "periodic")
    assert np.max(np.abs(ref - got)) < 1e-12


def test_sine_modes_closed_form():
    """sin(2 pi x) sin(2 pi y) on a periodic grid is a sum of the four modes
    k = (+-1, +-1); each is scaled by its eigenvalue lambda(k) per step."""
    n = 48
    w = si.normalised_weights(25, seed=41)
    offs = core.offsets("box", 2, 2)
    y = np.arange(n)[:, None] / n
    x = np.arange(n)[None, :] / n
    u0 = np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
    steps = 40
    ref = np.zeros((n, n), dtype=np.complex128)
    # sin a sin b = -(1/4) sum_{s,t=+-1} s t e^{i(s a + t b)}
    for sy, sx in itertools.product((1, -1), repeat=2):
        lam = sum(w[k] * np.exp(2j * np.pi * (sy * o[0] + sx * o[1]) / n) for k, o in enumerate(offs))
        ref += -0.25 * sy * sx * lam ** steps * np.exp(2j * np.pi * (sy * y * n + sx * x * n) / n)
    got = core.run("box", 2, 2, w, u0, steps, "periodic")
    assert np.max(np.abs(ref.real - got)) < 1e-13
    assert np.max(np.abs(ref.imag)) < 1e-13


@pytest.mark.parametrize("shape,d,r", [("box", 2, 2), ("star", 2, 3), ("box", 3, 1), ("star", 3, 2)])
def test_constant_preserved(shape, d, r):
    dims = (17, 19) if d == 2 else (11, 12, 13)
    w = si.normalised_weights(model.K_points(shape, d, r), seed=51)
    u0 = np.full(dims, 0.625)
    for boundary, halo in (("periodic", 0.0), ("dirichlet", 0.625)):
        got = core.run(shape, d, r, w, u0, 7, boundary, halo)
        assert np.max(np.abs(got - 0.625)) < 1e-14
    # halo 0: only points at distance >= r*N from the boundary keep the constant
    N = 2
    got = core.run(shape, d, r, w, u0, N, "dirichlet", 0.0)
    inner = tuple(slice(r * N, n - r * N) for n in dims)
    assert np.max(np.abs(got[inner] - 0.625)) < 1e-14
    edge = got.copy()
    edge[inner] = 0.625
    assert np.min(edge) < 0.625 - 1e-3


def _symmetric_weights(shape, d, r, seed):
    offs = core.offsets(shape, d, r)
    raw = si.dyadic_weights(len(offs), seed=seed)
    index = {tuple(o): k for k, o in enumerate(offs)}
    w = np.array([raw[min(k, index[tuple(-o)])] for k, o in enumerate(offs)])
    return w


@pytest.mark.parametrize("shape,d,r", [("box", 2, 1), ("star", 2, 2), ("box", 3, 1), ("star", 3, 2)])
def test_linear_field_exact(shape, d, r):
    """Symmetric weights map a + b.x to (sum w)(a + b.x): exact with dyadic data."""
    dims = (20, 22) if d == 2 else (12, 11, 13)
    w = _symmetric_weights(shape, d, r, seed=61)
    coords = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in dims], indexing="ij")
    coef = [3.0, -2.0, 5.0][:d]
    u0 = 7.0 + sum(c * g for c, g in zip(coef, coords))
    N = 2
    got = core.run(shape, d, r, w, u0, N, "dirichlet")
    s = float(np.sum(w))
    inner = tuple(slice(r * N, n - r * N) for n in dims)
    assert np.array_equal(got[inner], (s ** N * u0)[inner])


def test_quadratic_growth():
    """x0^2 -> x0^2 + N * sum_o w[o] o_0^2 for symmetric weights summing to 1."""
    offs = core.offsets("box", 2, 2)
    w = _symmetric_weights("box", 2, 2, seed=71)
    w = w / w.sum()
    dims = (40, 16)
    x0 = np.arange(dims[0], dtype=np.float64)[:, None] * np.ones(dims)
    N = 3
    got = core.run("box", 2, 2, w, x0 ** 2, N, "dirichlet")
    m2 = float(np.sum(w * offs[:, 0] ** 2))
    inner = (slice(2 * N, dims[0] - 2 * N), slice(2 * N, dims[1] - 2 * N))
    assert np.max(np.abs(got[inner] - (x0 ** 2 + N * m2)[inner])) < 1e-11


def test_linearity_and_max_principle():
    w = si.normalised_weights(13, seed=81)
    a = si.uniform_grid((21, 23), seed=82)
    b = si.uniform_grid((21, 23), seed=83)
    fa = core.run("star", 2, 3, w, a, 5, "periodic")
    fb = core.run("star", 2, 3, w, b, 5, "periodic")
    fab = core.run("star", 2, 3, w, 2.0 * a - 3.0 * b, 5, "periodic")
    assert np.max(np.abs(fab - (2.0 * fa - 3.0 * fb))) < 1e-13
    assert fa.max() <= a.max() + 1e-15 and fa.min() >= a.min() - 1e-15


@pytest.mark.parametrize("shape,dims,r,boundary,steps", [
    ("box", (30, 27), 2, "dirichlet", 4), ("star", (30, 27), 3, "periodic", 5),
    ("box", (11, 9, 12), 1, "periodic", 3), ("star", (11, 12, 9), 2, "dirichlet", 3),
    ("box", (16, 16), 3, "periodic", 4)])
def test_window_bit_identical(shape, dims, r, boundary, steps):
    d = len(dims)
    w = si.normalised_weights(model.K_points(shape, d, r), seed=91)
    u0 = si.uniform_grid(dims, seed=92)
    full = core.run(shape, d, r, w, u0, steps, boundary, 0.3)
    rng = np.random.default_rng(0)
    for _ in range(4):
        lo = [int(rng.integers(0, n - 1)) for n in dims]
        hi = [int(rng.integers(l + 1, n + 1)) for l, n in zip(lo, dims)]
        win = core.run_window(shape, d, r, w, u0, steps, lo, hi, boundary, 0.3)
        sl = tuple(slice(l, h) for l, h in zip(lo, hi))
        assert np.array_equal(win, full[sl])


@pytest.mark.parametrize("shape,d,r,t", [("box", 2, 1, 3), ("star", 2, 2, 2), ("box", 3, 1, 2),
                                         ("star", 3, 1, 3), ("star", 2, 1, 4)])
def test_composite_equals_t_steps(shape, d, r, t):
    dims = (19, 23) if d == 2 else (9, 10, 11)
    K = model.K_points(shape, d, r)
    w = si.dyadic_weights(K, seed=101)
    u0 = si.dyadic_grid(dims, seed=102)
    Wc = compose.composite(shape, d, r, w, t)
    once = compose.apply_composite_periodic(Wc, u0)
    steps = core.run(shape, d, r, w, u0, t, "periodic")
    assert np.array_equal(once, steps)


def test_composite_fusion_example(golden):
    """Box-2D1R fused over 3 steps: 7x7 = 49 points vs 3 x 9 = 27 sequential."""
    ex = golden["fusion_example"]
    assert compose.support_size("box", 2, 1, 3) == ex["fused_points"]
    assert 3 * core.num_points("box", 2, 1) == ex["sequential_ops"]
    assert ex["fused_points"] - ex["sequential_ops"] == ex["redundant_ops"]


@pytest.mark.parametrize("shape,d,r,t", [(s, d, r, t) for s in ("box", "star") for d in (2, 3)
                                         for r in (1, 2, 3) for t in (1, 2, 3, 4)
                                         if not (d == 3 and r * t > 6)])
def test_support_size_closed_form(shape, d, r, t):
    """Box: (2rt+1)^d (paper, redundancy-factor section).  Star: the reading
    #{x : sum_i ceil(|x_i|/r) <= t}.  Both against the nonzero count of the
    explicitly composed kernel."""
    assert compose.support_size(shape, d, r, t) == model.K_fused(shape, d, r, t)


def test_window_dirichlet_corner_cone():
    """Window touching a corner with many steps (cone clipped by the grid)."""
    w = si.normalised_weights(49, seed=111)
    u0 = si.uniform_grid((25, 25), seed=112)
    full = core.run("box", 2, 3, w, u0, 9, "dirichlet")
    win = core.run_window("box", 2, 3, w, u0, 9, (0, 20), (3, 25), "dirichlet")
    assert np.array_equal(win, full[0:3, 20:25])
