"""Autotuner: candidates ranked by the model are timed; the chosen (path, T,
rows) is applied and cached; results after tuning still match the oracle."""
import numpy as np
import pytest

import stencil_inputs as si
from gpu_util import case_inputs, lowp_bound, oracle, rel_inf, run_gpu
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


@pytest.mark.parametrize("shape,d,r,dt,dims", [("box", 2, 3, "f32", (1024, 1536)),
                                               ("star", 3, 2, "f64", (64, 64, 96)),
                                               ("box", 2, 2, "bf16", (512, 2048))])
def test_autotune_applies_and_caches(stl, shape, d, r, dt, dims):
    import torch
    u0, u0r, t, w = case_inputs(shape, d, r, dims, dt, seed=8000 + r)
    p = stl.Plan(shape, d, r, w, dims, T=1, dtype=dt, boundary="periodic")
    x = t.cuda()
    y = torch.empty_like(x)
    g = p.autotune(x, y, 8, max_candidates=3)
    i = p.info()
    assert g > 0 and 1 <= i["T"] <= 4 and i["path_name"] in ("valu", "mfma")
    # same problem again: cached choice, no timing
    p2 = stl.Plan(shape, d, r, w, dims, T=1, dtype=dt, boundary="periodic")
    assert p2.autotune(x, y, 8) == g
    assert (p2.info()["T"], p2.info()["path"]) == (i["T"], i["path"])
    got = run_gpu(p, t, 6)
    if dt in ("f64", "f32"):
        ref = oracle(shape, d, r, w, u0, 6, "periodic")
        assert rel_inf(got, ref) <= (1e-12 if dt == "f64" else 1e-5)
    else:
        # 16-bit storage: arithmetic error against the oracle on the rounded
        # data, within the bound of the slower of the two paths the tuner may
        # pick (MFMA: composite weights in bf16; VALU: float32 weights)
        T = p.info()["T"]
        ref = oracle(shape, d, r, w, u0r, 6, "periodic")
        err = float(np.max(np.abs(got - ref)))
        passes = -(-6 // T)
        assert err <= lowp_bound(dt, omodel.K_fused(shape, d, r, T), passes, float(np.max(np.abs(u0r))))
