"""GPU parity of the VALU path (temporal fusion) against the FP64 oracle.

Sizes span several workgroup bands and row segments with ragged tails; steps
are chosen so that the last pass has fewer than T steps.  Tolerances: FP64
relative max-norm error <= 1e-12, FP32 <= 1e-5 (inputs rounded to float32,
error measured against the oracle on the original float64 data)."""
import numpy as np
import pytest

import stencil_inputs as si
from gpu_util import case_inputs, oracle, rel_inf, run_gpu

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


def test_star2d1r_jacobi_512(stl):
    """Star-2D1R, weights 0.2, 512x512 FP64, U[0,1) seed 1001, zero Dirichlet
    halo, 10 steps, T = 1."""
    u0 = si.uniform_grid((512, 512), seed=si.data_seed(1, 1))
    w = np.full(5, 0.2)
    p = stl.Plan("star", 2, 1, w, (512, 512), T=1, dtype="f64", path="valu")
    got = run_gpu(p, si.round_to(u0, "f64")[1], 10)
    ref = oracle("star", 2, 1, w, u0, 10, "dirichlet")
    assert rel_inf(got, ref) <= 1e-12


CASES = [(shape, r, T, dt) for shape in ("star", "box") for r in (1, 2, 3) for T in (1, 2, 3, 4)
         for dt in ("f64", "f32")]


@pytest.mark.parametrize("shape,r,T,dt", CASES)
def test_valu2d_dirichlet(stl, shape, r, T, dt):
    dims = (301, 1213)
    u0, u0r, t, w = case_inputs(shape, 2, r, dims, dt, seed=2000 + 10 * r + T)
    steps = 2 * T + 1
    p = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="valu", halo=0.25)
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 2, r, w, u0, steps, "dirichlet", 0.25)
    assert rel_inf(got, ref) <= TOL[dt]


@pytest.mark.parametrize("shape,r,T,dt", [c for c in CASES if c[2] in (1, 3, 4)])
def test_valu2d_periodic(stl, shape, r, T, dt):
    dims = (157, 1100)
    u0, u0r, t, w = case_inputs(shape, 2, r, dims, dt, seed=3000 + 10 * r + T)
    steps = T + 2
    p = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, boundary="periodic", path="valu")
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 2, r, w, u0, steps, "periodic")
    assert rel_inf(got, ref) <= TOL[dt]


# the paper's evaluation patterns: r = 1 fused 5..8 deep, r = 7
CASES_EVAL = ([(shape, 1, T, dt) for shape in ("star", "box") for T in (5, 6, 7, 8) for dt in ("f64", "f32")]
              + [("box", 7, 1, "f64"), ("box", 7, 1, "f32"), ("star", 7, 1, "f32"), ("star", 7, 1, "f64")])


@pytest.mark.parametrize("shape,r,T,dt", CASES_EVAL)
@pytest.mark.parametrize("boundary", ["dirichlet", "periodic"])
def test_valu2d_eval_patterns(stl, shape, r, T, dt, boundary):
    """Deep fusion and radius 7 over several column bands and row segments
    with ragged edges; steps = T + 3 adds a remainder pass."""
    dims = (203, 1000)
    u0, u0r, t, w = case_inputs(shape, 2, r, dims, dt, seed=2600 + 10 * r + T)
    steps = T + 3
    p = stl.Plan(shape, 2, r, w, dims, T=T, dtype=dt, path="valu", boundary=boundary, halo=0.25)
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 2, r, w, u0, steps, boundary, 0.25)
    assert rel_inf(got, ref) <= TOL[dt]


@pytest.mark.parametrize("dims", [(1, 1), (1, 7), (9, 1), (5, 3), (33, 2049), (2, 513)])
def test_valu2d_small_and_thin(stl, dims):
    for boundary in ("dirichlet", "periodic"):
        u0, u0r, t, w = case_inputs("box", 2, 2, dims, "f64", seed=4000)
        p = stl.Plan("box", 2, 2, w, dims, T=3, dtype="f64", path="valu", boundary=boundary)
        got = run_gpu(p, t, 7)
        ref = oracle("box", 2, 2, w, u0, 7, boundary)
        assert rel_inf(got, ref) <= 1e-12, (dims, boundary)


def test_valu2d_t_fusion_consistent(stl):
    """T-fused passes equal single-step passes (both against the oracle and
    against each other)."""
    dims = (400, 900)
    u0, u0r, t, w = case_inputs("box", 2, 3, dims, "f64", seed=4100)
    outs = []
    for T in (1, 2, 4):
        p = stl.Plan("box", 2, 3, w, dims, T=T, dtype="f64", path="valu")
        outs.append(run_gpu(p, t, 8))
    ref = oracle("box", 2, 3, w, u0, 8, "dirichlet")
    for o in outs:
        assert rel_inf(o, ref) <= 1e-12
    assert rel_inf(outs[0], outs[2]) <= 1e-13


def test_steps_zero_copies(stl):
    import torch
    dims = (64, 80)
    u0, u0r, t, w = case_inputs("star", 2, 1, dims, "f32", seed=4200)
    p = stl.Plan("star", 2, 1, w, dims, T=2, dtype="f32")
    got = run_gpu(p, t, 0)
    assert np.array_equal(got, u0r)


def test_in_not_modified_and_alias_rejected(stl):
    import torch
    dims = (128, 256)
    u0, u0r, t, w = case_inputs("box", 2, 1, dims, "f64", seed=4300)
    p = stl.Plan("box", 2, 1, w, dims, T=2, dtype="f64")
    x = t.cuda()
    y = torch.empty_like(x)
    p.run(x, y, 5)
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), u0r)
    with pytest.raises(stl.StencilError) as e:
        p.run(x, x, 3)
    assert e.value.status == "ALIAS"


CASES3 = [(shape, r, T, dt) for shape in ("star", "box") for r in (1, 2, 3) for T in (1, 2, 3)
          for dt in ("f64", "f32")]


@pytest.mark.parametrize("shape,r,T,dt", CASES3)
@pytest.mark.parametrize("boundary", ["dirichlet", "periodic"])
def test_valu3d(stl, shape, r, T, dt, boundary):
    """3D sweeps over several in-plane tiles with ragged edges; combinations
    without a fused kernel run as single-step passes (same result)."""
    if shape == "box" and r == 3 and T > 1:
        pytest.skip("covered by T = 1 (same single-step passes)")
    dims = (19, 41, 75) if r < 3 else (13, 29, 40)
    u0, u0r, t, w = case_inputs(shape, 3, r, dims, dt, seed=5000 + 10 * r + T)
    steps = T + 1
    p = stl.Plan(shape, 3, r, w, dims, T=T, dtype=dt, path="valu", boundary=boundary, halo=0.5)
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 3, r, w, u0, steps, boundary, 0.5)
    assert rel_inf(got, ref) <= TOL[dt]


FUSED3 = [("star", 1, 2), ("star", 1, 3), ("star", 2, 2), ("star", 2, 3), ("star", 3, 2), ("box", 1, 2),
          ("box", 1, 3)]


@pytest.mark.parametrize("shape,r,T", FUSED3)
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("boundary", ["dirichlet", "periodic"])
@pytest.mark.parametrize("dims", [(21, 150, 144), (17, 131, 141)])
def test_valu3d_fused_many_tiles(stl, shape, r, T, dt, boundary, dims):
    """Fused 3D passes (T >= 2) over several in-plane tiles of the largest
    thread layouts, with ragged edges, rows whose length is and is not a
    whole number of vectors, and a remainder pass (2T + 1 steps)."""
    u0, u0r, t, w = case_inputs(shape, 3, r, dims, dt, seed=5700 + 10 * r + T + dims[2])
    steps = 2 * T + 1
    p = stl.Plan(shape, 3, r, w, dims, T=T, dtype=dt, path="valu", boundary=boundary, halo=0.5)
    assert p.info()["T_fused"] == T
    got = run_gpu(p, t, steps)
    ref = oracle(shape, 3, r, w, u0, steps, boundary, 0.5)
    assert rel_inf(got, ref) <= TOL[dt]


@pytest.mark.parametrize("dims", [(1, 1, 1), (3, 5, 7), (2, 9, 70), (9, 17, 3)])
@pytest.mark.parametrize("shape,r", [("star", 2), ("box", 1), ("star", 3)])
@pytest.mark.parametrize("boundary", ["dirichlet", "periodic"])
def test_valu3d_one_step_small_grids(stl, dims, shape, r, boundary):
    """One-step 3D passes stage the plane halo around the tile: grids smaller
    than the halo (a periodic halo wraps several times; a Dirichlet one is
    mostly h) and thinner than one tile in every direction."""
    u0, u0r, t, w = case_inputs(shape, 3, r, dims, "f64", seed=5300 + 10 * r + sum(dims))
    p = stl.Plan(shape, 3, r, w, dims, T=1, dtype="f64", path="valu", boundary=boundary, halo=0.375)
    got = run_gpu(p, t, 3)
    ref = oracle(shape, 3, r, w, u0, 3, boundary, 0.375)
    assert rel_inf(got, ref) <= 1e-12


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("r", [2, 3])
def test_valu3d_large_box_many_tiles(stl, r, dt):
    """Boxes with r >= 2 run on the one-step kernel: several in-plane tiles and
    plane segments with ragged edges, Dirichlet halo h = 0.25, two steps."""
    dims = (37, 70, 133)
    u0, u0r, t, w = case_inputs("box", 3, r, dims, dt, seed=5200 + r)
    p = stl.Plan("box", 3, r, w, dims, T=1, dtype=dt, path="valu", boundary="dirichlet", halo=0.25)
    got = run_gpu(p, t, 2)
    ref = oracle("box", 3, r, w, u0, 2, "dirichlet", 0.25)
    assert rel_inf(got, ref) <= TOL[dt]


def test_3d_periodic_patterns_reduced(stl):
    """Star-3D2R and Box-3D1R, periodic, T = 3 with a remainder pass (50 steps
    at full size; 8 steps here on 64^3)."""
    for shape, r in (("star", 2), ("box", 1)):
        dims = (64, 64, 64)
        u0, u0r, t, w = case_inputs(shape, 3, r, dims, "f64", seed=5500 + r)
        p = stl.Plan(shape, 3, r, w, dims, T=3, dtype="f64", path="valu", boundary="periodic")
        got = run_gpu(p, t, 8)
        ref = oracle(shape, 3, r, w, u0, 8, "periodic")
        assert rel_inf(got, ref) <= 1e-12
