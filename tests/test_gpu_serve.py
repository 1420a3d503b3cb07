"""Served stream on the GPU: jobs of mixed shape, d, r, size, steps and
boundary arrive while others run; every result equals the same job run alone
(bitwise: same plan, same kernels) and matches the FP64 oracle (FP32
tolerance)."""
import time

import numpy as np
import pytest

import stencil_inputs as si
from gpu_util import oracle, rel_inf
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


def _trace(n=24):
    tr = si.served_trace(n, seed=5000, rate_per_s=400.0, side2d=(64, 700), side3d=(16, 48),
                         steps=(1, 12))
    jobs = []
    for t in tr:
        K = omodel.K_points(t["shape"], t["d"], t["r"])
        w = si.normalised_weights(K, t["weight_seed"])
        u0 = si.uniform_grid(t["dims"], t["data_seed"])
        jobs.append((t, w, u0))
    return jobs


def test_served_mix_equals_alone_and_oracle(stl):
    import torch
    from paper_2603_00477_amd.serve import GpuExecutor, Job, StencilServer, latency_stats

    ex = GpuExecutor()
    srv = StencilServer(ex, hbm_budget=64 << 20).start()
    trace = _trace()
    futs = []
    t0 = time.perf_counter()
    for t, w, u0 in trace:
        now = time.perf_counter() - t0
        if t["arrival"] > now:
            time.sleep(t["arrival"] - now)
        job = Job(t["shape"], t["d"], t["r"], w, t["dims"], t["steps"], dtype="f32",
                  boundary=t["boundary"], data=torch.from_numpy(u0.astype(np.float32)), id=t["id"])
        futs.append((job, srv.submit(job)))
    results = [(job, f.result(timeout=120)) for job, f in futs]
    srv.stop()
    assert srv.rounds < sum(-(-j.steps // 1) for j, _ in results)  # rounds were shared
    st = latency_stats(srv.done)
    assert st["n"] == len(trace) and st["p99_ms"] >= st["p50_ms"] > 0
    for (job, d), (t, w, u0) in zip(results, trace):
        served = d.output.cpu()
        # alone, same plan choice
        st_alone = ex.prepare(job)
        left = job.steps
        while left > 0:
            s = ex.pass_steps(st_alone, left)
            ex.wait(ex.run_round([st_alone], [s]))
            left -= s
        alone = ex.result(st_alone).cpu()
        ex.release(st_alone)
        assert torch.equal(served, alone), t
        ref = oracle(t["shape"], t["d"], t["r"], w, u0, t["steps"], t["boundary"])
        assert rel_inf(served.to(torch.float64).numpy(), ref) <= 1e-5, t
