"""Batched runs: many grids of uneven size (and mixed variants) in one
stencil_run_batch call give exactly the result of running each job alone,
and match the oracle."""
import numpy as np
import pytest

import stencil_inputs as si
from gpu_util import case_inputs, oracle, rel_inf
from oracle import model as omodel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def stl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_00477_amd as stl
    stl.lib()
    return stl


def _jobs():
    rng = np.random.default_rng(0)
    jobs = []
    # same variant (box-2D r2 T2 f32), uneven sizes -> one batched launch per round
    for i in range(6):
        dims = (int(rng.integers(20, 700)), int(rng.integers(20, 1500)))
        jobs.append(("box", 2, 2, 2, "f32", dims, int(rng.integers(1, 9)), "dirichlet" if i % 2 else "periodic"))
    # other variants mixed in, including MFMA and 3D
    jobs += [("star", 2, 1, 3, "f64", (300, 410), 7, "dirichlet"),
             ("star", 2, 1, 3, "f64", (33, 2000), 4, "periodic"),
             ("box", 3, 1, 2, "f32", (20, 40, 70), 5, "periodic"),
             ("star", 3, 2, 1, "f64", (17, 30, 50), 3, "dirichlet"),
             ("box", 2, 3, 1, "f64", (100, 120), 0, "dirichlet")]
    return jobs


def test_batch_equals_alone(stl):
    import torch
    jobs = _jobs()
    plans, ins, outs_b, outs_a, refs = [], [], [], [], []
    for k, (shape, d, r, T, dt, dims, steps, bnd) in enumerate(jobs):
        u0, u0r, t, w = case_inputs(shape, d, r, dims, dt, seed=7000 + k)
        path = "mfma" if (k == 6) else "valu"
        p = stl.Plan(shape, d, r, w, dims, T=T, dtype=dt, boundary=bnd, path=path)
        plans.append(p)
        x = t.cuda()
        ins.append(x)
        outs_b.append(torch.empty_like(x))
        outs_a.append(torch.empty_like(x))
        refs.append((shape, d, r, w, u0, steps, bnd, dt))
    stl.run_batch(plans, ins, outs_b, [j[6] for j in jobs])
    torch.cuda.synchronize()
    for p, x, y, j in zip(plans, ins, outs_a, jobs):
        p.run(x, y, j[6])
    torch.cuda.synchronize()
    for k in range(len(jobs)):
        a = outs_a[k].cpu()
        b = outs_b[k].cpu()
        assert torch.equal(a, b), jobs[k]
        shape, d, r, w, u0, steps, bnd, dt = refs[k]
        ref = oracle(shape, d, r, w, u0, steps, bnd)
        tol = 1e-12 if dt == "f64" else 1e-5
        assert rel_inf(b.to(torch.float64).numpy(), ref) <= tol, jobs[k]


def test_batch_repeated_calls_reuse_staging(stl):
    """Back-to-back batch calls (the job table staging is reused)."""
    import torch
    w = si.normalised_weights(13, 1)
    plans, ins, outs = [], [], []
    for k in range(12):
        dims = (64 + 13 * k, 200 + 7 * k)
        plans.append(stl.Plan("star", 2, 3, w, dims, T=1, dtype="f32"))
        ins.append(torch.rand(dims, device="cuda", dtype=torch.float32))
        outs.append(torch.empty_like(ins[-1]))
    ref = []
    for p, x in zip(plans, ins):
        y = torch.empty_like(x)
        p.run(x, y, 3)
        ref.append(y)
    for _ in range(5):
        stl.run_batch(plans, ins, outs, [3] * 12)
    torch.cuda.synchronize()
    for a, b in zip(ref, outs):
        assert torch.equal(a, b)


def test_batch_argument_errors(stl):
    import torch
    w = si.normalised_weights(9, 1)
    p = stl.Plan("box", 2, 1, w, (32, 32), T=1, dtype="f32")
    x = torch.rand(32, 32, device="cuda")
    with pytest.raises(stl.StencilError) as e:
        stl.run_batch([p, p], [x, x], [torch.empty_like(x), torch.empty_like(x)], [1, 1])
    assert e.value.status == "INVALID_ARG"
    with pytest.raises(stl.StencilError) as e:
        stl.run_batch([p], [x], [x], [1])
    assert e.value.status == "ALIAS"


def test_batch_job_tables_beyond_staging_capacity(stl):
    """Job tables larger than the staging slot's initial 64 KiB: the slot
    grows while tables staged earlier in the same call are still to be read
    (a float64 Box-2D3R job entry carries its 49 weights, so 150 jobs of a
    variant stage about 70 KiB).  Two variants, two calls in a row; every
    result equals the job run alone, bit for bit."""
    import torch
    w = si.normalised_weights(49, 3)
    plans, ins, outs, steps = [], [], [], []
    for k in range(300):
        dims = (16 + (k % 7), 20 + (k * 13) % 61)
        T = 1 if k < 150 else 2
        plans.append(stl.Plan("box", 2, 3, w, dims, T=T, dtype="f64", path="valu"))
        g = torch.Generator(device="cuda")
        g.manual_seed(9000 + k)
        ins.append(torch.rand(dims, generator=g, device="cuda", dtype=torch.float64))
        outs.append(torch.empty_like(ins[-1]))
        steps.append(T)
    ref = []
    for p, x, s in zip(plans, ins, steps):
        y = torch.empty_like(x)
        p.run(x, y, s)
        ref.append(y)
    for _ in range(2):
        for o in outs:
            o.fill_(float("nan"))
        stl.run_batch(plans, ins, outs, steps)
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(ref, outs)):
            assert torch.equal(a, b), k


def test_batch_groups_3d_and_mfma(stl):
    """Several jobs per variant, so that 3D VALU passes (fused star/box
    kernel and the one-step large-box kernel) and 2D MFMA passes (float32,
    bf16, compensated; Dirichlet ones with their boundary-band fix-up) go
    out as batched launches: every result equals the job run alone, bit for
    bit, and matches the oracle."""
    import torch
    from gpu_util import lowp_bound
    rng = np.random.default_rng(11)
    spec = ([("star", 3, 2, 2, "f32", "valu", b) for b in ("periodic", "dirichlet", "periodic")]
            + [("box", 3, 1, 1, "f64", "valu", b) for b in ("dirichlet", "periodic")]
            + [("box", 3, 2, 1, "f32", "valu", b) for b in ("periodic", "dirichlet")]
            + [("box", 2, 2, 2, "f32", "mfma", b) for b in ("dirichlet", "dirichlet", "periodic")]
            + [("box", 2, 2, 4, "bf16", "mfma", "periodic")] * 2
            + [("star", 2, 1, 3, "bf16x3", "mfma", b) for b in ("periodic", "dirichlet")])
    plans, ins, outs_b, outs_a, refs, steps = [], [], [], [], [], []
    for k, (shape, d, r, T, dt, path, bnd) in enumerate(spec):
        if d == 3:
            dims = tuple(int(x) for x in rng.integers(12, 60, size=3))
        else:
            dims = (int(rng.integers(40, 300)), int(rng.integers(40, 500)))
        u0, u0r, t, w = case_inputs(shape, d, r, dims, dt, seed=7500 + k)
        p = stl.Plan(shape, d, r, w, dims, T=T, dtype=dt, boundary=bnd, path=path)
        plans.append(p)
        x = t.cuda()
        ins.append(x)
        outs_b.append(torch.empty_like(x))
        outs_a.append(torch.empty_like(x))
        steps.append(int(rng.integers(1, 10)))
        refs.append((shape, d, r, w, u0, u0r, bnd, dt, T))
    for _ in range(2):  # a second call reuses the staging ring
        stl.run_batch(plans, ins, outs_b, steps)
    torch.cuda.synchronize()
    for p, x, y, s in zip(plans, ins, outs_a, steps):
        p.run(x, y, s)
    torch.cuda.synchronize()
    for k in range(len(spec)):
        a, b = outs_a[k].cpu(), outs_b[k].cpu()
        assert torch.equal(a, b), spec[k]
        shape, d, r, w, u0, u0r, bnd, dt, T = refs[k]
        got = b.to(torch.float64).numpy()
        if dt in ("f64", "f32"):
            ref = oracle(shape, d, r, w, u0, steps[k], bnd)
            assert rel_inf(got, ref) <= (1e-12 if dt == "f64" else 1e-5), spec[k]
        else:
            ref = oracle(shape, d, r, w, u0r, steps[k], bnd)
            bound = lowp_bound(dt, omodel.K_fused(shape, d, r, T), -(-steps[k] // T), float(np.max(np.abs(u0r))))
            assert float(np.max(np.abs(got - ref))) <= bound, spec[k]
