"""stencil_run_noalloc: the allocation-free variant of stencil_run (its
intermediate grid lives in the library's static device array) gives exactly
the result of stencil_run, call after call on the same array, and refuses
what it cannot do without allocating."""
import numpy as np
import pytest

import stencil_inputs as si
from gpu_util import case_inputs, oracle, rel_inf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_00477_amd as stl
    stl.lib()
    return stl


def _pair(stl, shape, d, r, T, dt, dims, steps, path, seed, boundary="dirichlet"):
    import torch
    u0, u0r, t, w = case_inputs(shape, d, r, dims, dt, seed=seed)
    x = t.cuda()
    p = stl.Plan(shape, d, r, w, dims, T=T, dtype=dt, path=path, boundary=boundary)
    y_ref = torch.empty_like(x)
    p.run(x, y_ref, steps)
    y = torch.full_like(x, float("nan"))
    p.run_noalloc(x, y, steps)
    torch.cuda.synchronize()
    return p, x, y, y_ref, (shape, d, r, w, u0, steps, boundary, dt)


@pytest.mark.parametrize("path", ["valu", "mfma"])
def test_noalloc_equals_run_two_calls_second_smaller(stl, path):
    import torch
    # first call: 2000 x 2048 float64 (32 MiB, passes ping-pong through the
    # static array); second call: a smaller grid of another pattern
    calls = [("box", 2, 3, 2, "f64", (2000, 2048), 7), ("star", 2, 2, 4, "f32", (700, 901), 9)]
    for k, (shape, d, r, T, dt, dims, steps) in enumerate(calls):
        p, x, y, y_ref, ref_args = _pair(stl, shape, d, r, T, dt, dims, steps, path, 9100 + k)
        assert torch.equal(y, y_ref), (path, k)
        shape, d, r, w, u0, steps, bnd, dt = ref_args
        ref = oracle(shape, d, r, w, u0, steps, bnd)
        assert rel_inf(y.double().cpu().numpy(), ref) <= (1e-12 if dt == "f64" else 1e-5)
        p.close()


def test_noalloc_3d_and_one_pass(stl):
    import torch
    for k, (T, steps) in enumerate([(2, 5), (3, 3)]):  # five passes; one pass (no scratch)
        p, x, y, y_ref, _ = _pair(stl, "star", 3, 2, T, "f32", (40, 50, 300), steps, "valu", 9200 + k,
                                  boundary="periodic")
        assert torch.equal(y, y_ref)
        p.close()


def test_noalloc_refusals(stl):
    import torch
    # a multi-pass run over a grid larger than the static array
    n = 4200  # 4200^2 float32 = 67.3 MiB > 64 MiB
    w = si.normalised_weights(5, 1)
    p = stl.Plan("star", 2, 1, w, (n, n), T=1, dtype="f32", path="valu")
    x = torch.rand((n, n), device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(stl.StencilError) as e:
        p.run_noalloc(x, y, 2)
    assert e.value.status == "INVALID_ARG" and "static scratch" in str(e.value)
    # ... while one pass needs no intermediate grid
    p.run_noalloc(x, y, 1)
    y_ref = torch.empty_like(x)
    p.run(x, y_ref, 1)
    torch.cuda.synchronize()
    assert torch.equal(y, y_ref)
    p.close()
    # an MFMA plan that never ran has no operand fragments on the device
    w = si.normalised_weights(9, 2)
    q = stl.Plan("box", 2, 1, w, (64, 64), T=2, dtype="f32", path="mfma")
    a = torch.rand((64, 64), device="cuda")
    b = torch.empty_like(a)
    with pytest.raises(stl.StencilError) as e:
        q.run_noalloc(a, b, 4)
    assert e.value.status == "UNSUPPORTED"
    q.close()
