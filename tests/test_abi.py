"""Host-side checks of the C ABI (no GPU needed): exported symbols, argument
validation, plan descriptions, the composite kernel against the oracle's, and
the library's roofline model against the oracle's closed forms and the
paper's printed cases."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2603_00477_amd as stl
import stencil_inputs as si
from oracle import compose as ocompose
from oracle import model as omodel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "stencil.h")).read()
    names = set(re.findall(r"^(?:int|void|double|const char \*)\s*\*?\s*(stencil_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 11
    L = ctypes.CDLL(stl._abi.LIB_PATH)
    for n in sorted(names):
        assert hasattr(L, n), n


@pytest.mark.parametrize("kw,status", [
    (dict(d=1), "INVALID_ARG"), (dict(d=4), "INVALID_ARG"), (dict(r=0), "INVALID_ARG"),
    (dict(T=0), "INVALID_ARG"), (dict(dtype=9), "INVALID_ARG"), (dict(boundary=7), "INVALID_ARG"),
    (dict(shape=5), "INVALID_ARG"), (dict(dims=(0, 5)), "INVALID_ARG"),
    (dict(weights=[float("nan")] * 9), "INVALID_ARG"),
])
def test_plan_validation(kw, status):
    args = dict(shape="box", d=2, r=1, weights=[1 / 9] * 9, dims=(16, 16), T=1, dtype="f64",
                boundary="dirichlet")
    args.update(kw)
    if args["d"] in (2, 3) and "dims" not in kw:
        args["dims"] = (16,) * args["d"]
    with pytest.raises(stl.StencilError) as e:
        stl.Plan(**args)
    assert e.value.status == status
    assert len(str(e.value)) > 20


def test_periodic_mfma_needs_room():
    w = [1 / 9] * 9
    with pytest.raises(stl.StencilError) as e:
        stl.Plan("box", 2, 1, w, (6, 64), T=3, dtype="f64", boundary="periodic", path="mfma")
    assert e.value.status == "INVALID_ARG"


def test_dirichlet_mfma_needs_a_band_kernel():
    # Box-3D1R fused 7 deep exists on the matrix path only: a Dirichlet plan
    # would have no kernel for its boundary band, a periodic one is accepted
    w = [1 / 27] * 27
    with pytest.raises(stl.StencilError) as e:
        stl.Plan("box", 3, 1, w, (32, 32, 32), T=7, dtype="f32", boundary="dirichlet", path="mfma")
    assert e.value.status == "UNSUPPORTED" and "boundary band" in str(e.value)
    p = stl.Plan("box", 3, 1, w, (32, 32, 32), T=7, dtype="f32", boundary="periodic", path="mfma")
    assert p.info()["path_name"] == "mfma"
    # the model predicts the vector units for this case; without a fused VALU
    # kernel of depth 7 the automatic choice still runs it there (T = 1 passes)
    assert stl.Plan("box", 3, 1, w, (32, 32, 32), T=7, dtype="f32", boundary="dirichlet").info()["path_name"] == "valu"


def test_bf16x3_is_mfma_only():
    with pytest.raises(stl.StencilError) as e:
        stl.Plan("box", 2, 2, [1 / 25] * 25, (64, 64), T=1, dtype="bf16x3", path="valu")
    assert e.value.status == "UNSUPPORTED"


def test_plan_info_fields():
    w = si.normalised_weights(49, 1)
    p = stl.Plan("box", 2, 3, w, (8192, 8192), T=2, dtype="f32")
    i = p.info()
    assert i["K"] == 49 and i["K_T"] == 169
    assert math.isclose(i["alpha"], 169 / 98)
    assert math.isclose(i["S"], 13 / 28)  # (2R+1) / Kp, R = 6, Kp = 28
    assert i["workspace_bytes"] >= 8192 * 8192 * 4
    assert i["path_name"] in ("valu", "mfma")
    p.set(stl._abi.OPT_HALO_VALUE, 0.5)
    assert p.info()["halo"] == 0.5
    p.set(stl._abi.OPT_T, 4)
    assert p.info()["T"] == 4 and p.info()["K_T"] == 625
    with pytest.raises(stl.StencilError):
        p.set(stl._abi.OPT_T, 0)
    with pytest.raises(stl.StencilError):
        p.set(99, 1.0)


@pytest.mark.parametrize("shape,d,r,T", [("box", 2, 1, 3), ("star", 2, 3, 2), ("box", 3, 1, 3),
                                         ("star", 3, 2, 3), ("box", 2, 3, 4), ("star", 2, 1, 5)])
def test_compose_matches_oracle(shape, d, r, T):
    K = omodel.K_points(shape, d, r)
    w = si.normalised_weights(K, seed=7)
    got, kt = stl.compose(shape, d, r, w, T)
    ref = ocompose.composite(shape, d, r, w, T)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) <= 1e-15 * np.max(np.abs(ref)) * T
    assert kt == omodel.K_fused(shape, d, r, T) == np.count_nonzero(ref)


def test_compose_dyadic_bit_exact():
    w = si.dyadic_weights(25, seed=3)
    got, _ = stl.compose("box", 2, 2, w, 3)
    assert np.array_equal(got, ocompose.composite("box", 2, 2, w, 3))


@pytest.mark.parametrize("shape,d,r,T,dt", [(s, d, r, T, dt) for s in ("box", "star") for d in (2, 3)
                                            for r in (1, 2, 3) for T in (1, 2, 4)
                                            for dt in ("f64", "f32", "bf16", "bf16x3")
                                            if not (d == 3 and r * T > 6)])
def test_model_matches_oracle(shape, d, r, T, dt):
    m = stl.model_predict(shape, d, r, T, dt)
    hw = stl.hw_default(dt)
    K = omodel.K_points(shape, d, r)
    D = {"f64": 8, "f32": 4, "bf16": 2, "bf16x3": 4}[dt]
    a = omodel.alpha(shape, d, r, T)
    S = m["S"]
    g = 3.0 if dt == "bf16x3" else 1.0
    assert m["K"] == K and m["K_T"] == omodel.K_fused(shape, d, r, T)
    assert math.isclose(m["alpha"], a)
    assert math.isclose(m["I_valu"], omodel.I_cu(K, D, T))
    assert math.isclose(m["I_mfma"], g * omodel.I_tc(K, D, T, a, S))
    assert math.isclose(m["P_valu"], omodel.P_cu(hw["PP_valu"], hw["BB"], K, D, T))
    assert math.isclose(m["P_mfma"], omodel.P_tc_actual(hw["PP_mfma"], hw["BB"], K, D, T, g * a, S))
    assert m["scenario"] == omodel.scenario(hw["PP_valu"], hw["PP_mfma"], hw["BB"], K, D, T, g * a, S)
    assert math.isclose(m["ratio"], omodel.speedup(hw["PP_valu"], hw["PP_mfma"], hw["BB"], K, D, T, g * a, S))
    assert math.isclose(m["gst_valu"], omodel.gstencils(m["P_valu"], K))
    assert m["sweet_spot"] == int(omodel.sweet_spot(hw["PP_valu"], hw["PP_mfma"], g * a, S))
    assert 0 < S <= 1


def test_library_model_reproduces_table3(golden):
    """The library's model with the paper's A100 ceilings and S reproduces the
    printed intensities, scenarios and changes of Table 3."""
    p = golden["a100_peaks"]
    for c in golden["table3"]["cases"]:
        dt = "f64" if c["dtype"] == "double" else "f32"
        PPtc = p["PP_tc_f64"] if dt == "f64" else (p["PP_tc_f32_sparse_inferred"] if c["sparse"]
                                                   else p["PP_tc_f32_dense_inferred"])
        PPcu = p["PP_cu_f64"] if dt == "f64" else p["PP_cu_f32_inferred"]
        hw = dict(BB=p["BB_inferred"], PP_valu=PPcu, PP_mfma=PPtc, PP_mfma_sparse=PPtc)
        m = stl.model_predict(c["shape"], c["d"], c["r"], c["t"], dt, S=c["S"], hw=hw)
        assert abs(m["I_mfma"] - c["tc"]["I"]) <= 0.005 * c["tc"]["I"]
        assert m["scenario"] == c["scenario"]
        assert {-1: "down", 0: "tie", 1: "up"}[m["winner"]] == c["change"]


@pytest.mark.parametrize("R,kdim", [(1, 4), (3, 4), (6, 4), (12, 4), (2, 32), (8, 32), (12, 32)])
def test_box_sparsity_closed_form(R, kdim):
    """Box layout: S = (2R+1)/Kp with Kp = 16 + 2R rounded up to the MFMA k."""
    dt = "f64" if kdim == 4 else "bf16"
    Kp = -(-(16 + 2 * R) // kdim) * kdim
    assert math.isclose(stl.mfma_sparsity("box", 2, R, 1, dt), (2 * R + 1) / Kp)
    assert math.isclose(stl.mfma_sparsity("box", 3, R, 1, dt), (2 * R + 1) / Kp) or R > 6


def test_auto_path_follows_model():
    w = si.normalised_weights(25, 2)
    p = stl.Plan("box", 2, 2, w, (1024, 1024), T=4, dtype="bf16")
    assert p.info()["predicted_winner"] == 1
    assert p.info()["path_name"] == "mfma"
    p2 = stl.Plan("box", 2, 3, si.normalised_weights(49, 2), (1024, 1024), T=1, dtype="f64")
    assert p2.info()["path_name"] == "valu"


def test_plan_info_reports_tile_rows_and_fused_depth():
    import paper_2603_00477_amd as stl
    w = [1.0 / 49] * 49
    p = stl.Plan("box", 2, 3, w, (64, 64), T=2, dtype="f64", path="valu", tile_rows=96)
    i = p.info()
    assert i["tile_rows"] == 96 and i["T_fused"] == 2
    # float64 Star-2D3R fused 5 deep has no kernel: a pass runs as one-step launches
    w13 = [1.0 / 13] * 13
    q = stl.Plan("star", 2, 3, w13, (64, 64), T=5, dtype="f64", path="valu")
    assert q.info()["T"] == 5 and q.info()["T_fused"] == 1


def test_sparse_path_model_and_availability():
    # Box-2D1R fused 7 deep in bf16: 15 kernel columns -> 8 column pairs of one
    # 16x16x64 instruction each; S = K_T / (64 * 8) against the sparse peak
    m = stl.model_predict("box", 2, 1, 7, "bf16", sparse=True)
    assert m["K_T"] == 225 and m["S"] == pytest.approx(225 / 512)
    dense = stl.model_predict("box", 2, 1, 7, "bf16")
    assert dense["S"] == pytest.approx(225 / (15 * 32))
    # same issued dense-equivalent work, twice the peak: the matrix ceiling doubles
    assert m["P_mfma_raw"] >= dense["P_mfma_raw"]
    assert stl.kernel_available("mfma_sparse", "bf16", "box", 2, 1, 7)
    assert stl.kernel_available("mfma_sparse", "f16", "star", 2, 2, 2)
    assert not stl.kernel_available("mfma_sparse", "bf16", "box", 2, 2, 4)   # composite radius 8
    assert not stl.kernel_available("mfma_sparse", "f32", "box", 2, 1, 1)
    p = stl.Plan("box", 2, 1, [1 / 9] * 9, (64, 64), T=7, dtype="bf16", path="mfma_sparse", boundary="periodic")
    i = p.info()
    assert i["path_name"] == "mfma_sparse" and i["S"] == pytest.approx(225 / 512)
    # Box-2D2R fused 3 deep: 13 columns, 7 pairs; switching to the dense path
    # gives the dense layout's S again
    q = stl.Plan("box", 2, 2, [1 / 25] * 25, (64, 64), T=3, dtype="bf16", path="mfma_sparse", boundary="periodic")
    assert q.info()["S"] == pytest.approx(169 / 448)
    q.set(stl._abi.OPT_PATH, stl.PATH_MFMA)
    assert q.info()["path_name"] == "mfma" and q.info()["S"] == pytest.approx(169 / 416)


def test_halo_model_terms():
    # float64 Box-2D3R fused 2 deep on 64 x 64 tiles: step 1 covers 80 x 80
    # (the needed 70 x 70 rounded up to 16-point tiles), step 2 64 x 64; each
    # 16 x 16 tile issues 7 columns x 6 four-deep k-blocks of 2*16*16*4 flops
    m = stl.model_predict("box", 2, 3, 2, "f64")
    assert m["C_mfma_seq"] == pytest.approx((25 + 16) * 7 * 6 * 2 * 16 * 16 * 4 / 4096)
    # it issues more than the kernel-fused layout (alpha / S = 1.72 / 0.464)
    assert m["C_mfma_seq"] > m["C_mfma"] and m["gst_mfma_seq"] < m["gst_mfma"]
    # VALU skirt: float64 bands at T = 2 are 256 columns (4 per lane); the
    # 6-column skirt rounds up to two whole lanes per side: 256 - 2*8 remain
    assert m["halo_valu"] == pytest.approx(256 / 240)
    # (the skirt rounds up to whole 16-byte vectors: 3 -> 4 columns)
    assert stl.model_predict("box", 2, 3, 1, "f64")["halo_valu"] == pytest.approx(128 / 120)
    # float64 r = 7 one-step passes run 4-column lanes: 256-column bands, 8-column skirts
    assert stl.model_predict("star", 2, 7, 1, "f64")["halo_valu"] == pytest.approx(256 / 240)
    # 3D one-step passes stage their halo: no skirt
    assert stl.model_predict("star", 3, 2, 1, "f32")["halo_valu"] == 1.0
    # 3D fused passes stage the input halo: float32 Star-3D2R T = 2 computes a
    # 64 x 64 layout for a 60 x 56 output tile (margin 2, left margin rounded
    # up to a 4-column vector); float64 Box-3D1R T = 2 a 32 x 64 layout for 30 x 60
    assert stl.model_predict("star", 3, 2, 2, "f32")["halo_valu"] == pytest.approx(4096 / (60 * 56))
    assert stl.model_predict("box", 3, 1, 2, "f64")["halo_valu"] == pytest.approx(2048 / (30 * 60))
    assert stl.kernel_available("mfma_seq", "bf16", "box", 2, 2, 4)
