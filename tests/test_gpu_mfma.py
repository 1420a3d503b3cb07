"""GPU parity of the MFMA path (kernel fusion as banded Toeplitz products)
against the FP64 oracle.

FP64 <= 1e-12 and FP32 <= 1e-5 relative max-norm error.  16-bit modes are
checked for arithmetic error (oracle run on the storage-rounded input, with
the float64 weights) against the worst-case bound of gpu_util.lowp_bound,
    passes * (u_store + u_w + K_T * 2^-24) * max|u0|
with u_store the storage unit roundoff (bf16 2^-8, f16 2^-11, float32 2^-24),
u_w the per-product operand error (bf16 2^-8, f16 2^-11, compensated hi/lo
split 3 * 2^-16: weight-split residual, data-split residual, dropped lo*lo)
and K_T * 2^-24 the float32 accumulation of K_T terms of a non-expansive
operator (weights >= 0, sum 1)."""
import numpy as np
import pytest

from gpu_util import U_STORE, case_inputs, lowp_bound, oracle, rel_inf, run_gpu
from oracle import model as omodel

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def stl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_00477_amd as stl
    stl.lib()
    return stl


CASES = [(shape, r, T, dt) for shape in ("star", "box") for r in (1, 2, 3) for T in (1, 2, 3, 4)
         for dt in ("f64", "f32")]


@pytest.mark.parametrize("shape,r,T,dt", CASES)
@pytest.mark.parametrize("boundary", ["dirichlet", "periodic"])
def test_mfma2d(stl, shape, r, T, dt, boundary):
    dims = (150, 217)
    u0, u0r, t, w = case_inputs(shape, 2, r, dims, dt, seed=6000 + 10 * r + T)
    steps = 2 * T + (1 if T > 1 else 0)
    p = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="mfma", boundary=boundary, halo=0.125)
    assert p.info()["path_name"] == "mfma"
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 2, r, w, u0, steps, boundary, 0.125)
    assert rel_inf(got, ref) <= TOL[dt]


@pytest.mark.parametrize("shape", ["box", "star"])
@pytest.mark.parametrize("r,T", [(1, 7), (7, 1)])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("boundary", ["dirichlet", "periodic"])
def test_mfma2d_radius7_composites(stl, shape, r, T, dt, boundary):
    """Composite radius 7 (the paper's Box/Star-2D1R fused 7 deep and
    Box/Star-2D7R): two full passes plus a remainder pass; Dirichlet adds the
    fix-up band."""
    dims = (150, 217)
    u0, u0r, t, w = case_inputs(shape, 2, r, dims, dt, seed=6500 + 10 * r + T + (shape == "star"))
    steps = 2 * T + 1
    p = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="mfma", boundary=boundary, halo=0.125)
    assert p.info()["path_name"] == "mfma"
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 2, r, w, u0, steps, boundary, 0.125)
    assert rel_inf(got, ref) <= TOL[dt]


@pytest.mark.parametrize("shape,r,T,dims", [("box", 1, 4, (17, 23)), ("star", 2, 2, (9, 70)),
                                            ("box", 7, 1, (15, 40)), ("box", 1, 7, (15, 15))])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_mfma2d_small_periodic(stl, shape, r, T, dims, dt):
    """Periodic grids smaller than one 64 x 64 tile, down to the minimum
    2rT + 1 points per axis: the staged block wraps more than once."""
    u0, u0r, t, w = case_inputs(shape, 2, r, dims, dt, seed=6700 + 10 * r + T)
    steps = 2 * T
    p = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="mfma", boundary="periodic")
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 2, r, w, u0, steps, "periodic")
    assert rel_inf(got, ref) <= TOL[dt]


def test_mfma_matches_valu_f64(stl):
    dims = (257, 300)
    u0, u0r, t, w = case_inputs("box", 2, 3, dims, "f64", seed=6100)
    outs = {}
    for path in ("valu", "mfma"):
        p = stl.Plan("box", 2, 3, w, dims, T=2, dtype="f64", path=path)
        outs[path] = run_gpu(p, t, 6)
    assert rel_inf(outs["mfma"], outs["valu"]) <= 1e-13


def _bound(dt, shape, d, r, T, steps, umax):
    KT = omodel.K_fused(shape, d, r, T)
    passes = -(-steps // T)
    return lowp_bound(dt, KT, passes, umax)


@pytest.mark.parametrize("dt", ["bf16", "f16", "bf16x3"])
@pytest.mark.parametrize("shape,r,T", [("box", 2, 1), ("box", 2, 2), ("box", 2, 4), ("star", 1, 3),
                                       ("box", 3, 2), ("star", 3, 1)])
@pytest.mark.parametrize("boundary", ["periodic", "dirichlet"])
def test_mfma2d_low_precision(stl, dt, shape, r, T, boundary):
    dims = (160, 300)
    u0, u0r, t, w = case_inputs(shape, 2, r, dims, dt, seed=6200 + 10 * r + T)
    steps = 2 * T
    p = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="mfma", boundary=boundary)
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 2, r, w, u0r, steps, boundary)
    err = float(np.max(np.abs(got - ref)))
    assert err <= _bound(dt, shape, 2, r, T, steps, float(np.max(np.abs(u0r)))), err


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("T", [1, 2, 4])
def test_valu2d_low_precision_storage(stl, dt, T):
    """VALU path on 16-bit storage with float32 arithmetic (intermediate steps
    of a pass kept in float32 on chip)."""
    dims = (130, 2100)
    u0, u0r, t, w = case_inputs("box", 2, 2, dims, dt, seed=6300 + T)
    steps = 2 * T + 1
    p = stl.Plan("box", 2, 2, w, dims, T=T, dtype=dt, path="valu", boundary="periodic")
    got = run_gpu(p, t, steps)
    ref = oracle("box", 2, 2, w, u0r, steps, "periodic")
    # per pass: one rounding to storage, T float32 steps of 25 float32-rounded
    # weights (products and sums within (25 + 1) 2^-24 per step)
    passes = -(-steps // T)
    err = float(np.max(np.abs(got - ref)))
    assert err <= passes * (U_STORE[dt] + 26 * T * 2.0 ** -24) * float(np.max(np.abs(u0r)))


CASES3 = [(shape, r, T, dt) for shape, r in (("star", 1), ("star", 2), ("box", 1)) for T in (1, 2, 3)
          for dt in ("f64", "f32")]


@pytest.mark.parametrize("shape,r,T,dt", CASES3)
@pytest.mark.parametrize("boundary", ["dirichlet", "periodic"])
def test_mfma3d(stl, shape, r, T, dt, boundary):
    dims = (23, 37, 70)
    u0, u0r, t, w = case_inputs(shape, 3, r, dims, dt, seed=6400 + 10 * r + T)
    steps = T + 1 if T > 1 else 2
    p = stl.Plan(shape, 3, r, w, dims, T=T, dtype=dt, path="mfma", boundary=boundary, halo=0.25)
    assert p.info()["path_name"] == "mfma"
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 3, r, w, u0, steps, boundary, 0.25)
    assert rel_inf(got, ref) <= TOL[dt]


def test_mfma3d_radius7_composite(stl):
    """Composite radius 7 in 3D (the paper's Box-3D1R fused 7 deep, float):
    two full passes and a one-step remainder on a periodic grid with ragged
    in-plane tiles and the minimum 2rT + 1 planes."""
    dims = (15, 37, 70)
    u0, u0r, t, w = case_inputs("box", 3, 1, dims, "f32", seed=6900)
    p = stl.Plan("box", 3, 1, w, dims, T=7, dtype="f32", path="mfma", boundary="periodic")
    assert p.info()["path_name"] == "mfma"
    got = run_gpu(p, t, 15)
    ref = oracle("box", 3, 1, w, u0, 15, "periodic")
    assert rel_inf(got, ref) <= TOL["f32"]


@pytest.mark.parametrize("shape,r,T,dims", [("box", 1, 3, (9, 11, 13)), ("star", 2, 2, (9, 20, 70))])
def test_mfma3d_small_periodic(stl, shape, r, T, dims):
    """Periodic 3D grids smaller than one in-plane tile."""
    u0, u0r, t, w = case_inputs(shape, 3, r, dims, "f64", seed=6800 + 10 * r + T)
    p = stl.Plan(shape, 3, r, w, dims, T=T, dtype="f64", path="mfma", boundary="periodic")
    got = run_gpu(p, t, 2 * T)
    ref = oracle(shape, 3, r, w, u0, 2 * T, "periodic")
    assert rel_inf(got, ref) <= 1e-12


SPARSE_CASES = [("box", 1, 1), ("box", 1, 4), ("box", 1, 7), ("box", 2, 3), ("box", 3, 2), ("star", 1, 3),
                ("star", 2, 2), ("star", 3, 1)]


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("shape,r,T", SPARSE_CASES)
@pytest.mark.parametrize("boundary", ["periodic", "dirichlet"])
def test_mfma2d_sparse(stl, dt, shape, r, T, boundary):
    """2:4 structured-sparse MFMA (one v_smfmac per pair of kernel columns):
    arithmetic error against the oracle on the rounded data within the same
    bound as the dense 16-bit kernels, over two full passes and a remainder
    pass; Dirichlet plans of depths without a fused 16-bit VALU kernel for
    the boundary band are refused."""
    dims = (150, 217)
    u0, u0r, t, w = case_inputs(shape, 2, r, dims, dt, seed=6600 + 10 * r + T)
    steps = 2 * T + 1
    if boundary == "dirichlet" and T > 4:
        with pytest.raises(stl.StencilError) as e:
            stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="mfma_sparse", boundary=boundary)
        assert e.value.status == "UNSUPPORTED"
        return
    p = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="mfma_sparse", boundary=boundary)
    assert p.info()["path_name"] == "mfma_sparse"
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 2, r, w, u0r, steps, boundary)
    err = float(np.max(np.abs(got - ref)))
    assert err <= _bound(dt, shape, 2, r, T, steps, float(np.max(np.abs(u0r)))), err
    # the dense kernel computes the same products (summed in another order)
    q = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="mfma", boundary=boundary)
    dense = run_gpu(q, t, steps)
    assert float(np.max(np.abs(dense - ref))) <= _bound(dt, shape, 2, r, T, steps, float(np.max(np.abs(u0r))))


def test_mfma2d_sparse_refusals(stl):
    w = si_weights = np.full(25, 1 / 25)
    # composite radius 8 does not fit the 2:4 layout; float32 has no sparse instruction
    for dt, r, T in (("bf16", 2, 4), ("f32", 1, 2)):
        with pytest.raises(stl.StencilError) as e:
            stl.Plan("box", 2, r, np.full((2 * r + 1) ** 2, 1.0 / (2 * r + 1) ** 2), (64, 64), T=T, dtype=dt,
                     path="mfma_sparse", boundary="periodic")
        assert e.value.status == "UNSUPPORTED"


SEQ_CASES = [(shape, r, T) for shape in ("box", "star") for r, T in ((1, 1), (1, 4), (2, 2), (2, 3), (3, 2), (3, 4))]


@pytest.mark.parametrize("shape,r,T", SEQ_CASES)
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("boundary", ["dirichlet", "periodic"])
def test_mfma2d_sequential(stl, shape, r, T, dt, boundary):
    """Sequential-step fusion on the matrix cores (T single-step band products
    per pass, intermediates in LDS): the oracle within 1e-12 / 1e-5 over two
    passes and a remainder, Dirichlet with a non-zero halo value and no
    boundary-band fix-up, on grids with ragged 64-point tiles."""
    dims = (150, 217)
    u0, u0r, t, w = case_inputs(shape, 2, r, dims, dt, seed=6850 + 10 * r + T)
    steps = 2 * T + 1
    p = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="mfma_seq", boundary=boundary, halo=0.125)
    assert p.info()["path_name"] == "mfma_seq"
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 2, r, w, u0, steps, boundary, 0.125)
    assert rel_inf(got, ref) <= TOL[dt]


@pytest.mark.parametrize("dt", ["bf16", "f16"])
@pytest.mark.parametrize("shape,r,T", [("box", 2, 4), ("star", 3, 2), ("box", 1, 3)])
def test_mfma2d_sequential_low_precision(stl, dt, shape, r, T):
    """16-bit sequential fusion: every step rounds its result to the storage
    type, so the bound counts steps rather than passes (single-step weights
    rounded once, K float32 accumulations per step)."""
    dims = (160, 300)
    u0, u0r, t, w = case_inputs(shape, 2, r, dims, dt, seed=6870 + 10 * r + T)
    steps = 2 * T + 1
    p = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="mfma_seq", boundary="periodic")
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 2, r, w, u0r, steps, "periodic")
    err = float(np.max(np.abs(got - ref)))
    K = omodel.K_points(shape, 2, r)
    assert err <= lowp_bound(dt, K, steps, float(np.max(np.abs(u0r)))), err


@pytest.mark.parametrize("dims", [(5, 7), (9, 70), (64, 64), (65, 129)])
def test_mfma2d_sequential_small_periodic(stl, dims):
    """Periodic grids smaller than the tile and its halo (the staged block
    wraps several times)."""
    u0, u0r, t, w = case_inputs("box", 2, 2, dims, "f64", seed=6890)
    p = stl.Plan("box", 2, 2, w, dims, T=3, dtype="f64", path="mfma_seq", boundary="periodic")
    got = run_gpu(p, t, 7)
    ref = oracle("box", 2, 2, w, u0, 7, "periodic")
    assert rel_inf(got, ref) <= 1e-12
