"""MI355X-native explicit stencil sweeps (box/star, d = 2 or 3, radius r,
T steps fused per pass) with a VALU and an MFMA kernel family and the
roofline model of arXiv 2603.00477 that predicts which one wins.

Python binding of the C ABI (include/stencil.h).  PyTorch provides device
memory and streams; every arithmetic step runs in the HIP library.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import (BF16, BOX, DIRICHLET, F16, F32, F32_BF16X3, F64, PATH_AUTO, PATH_MFMA,
                   PATH_MFMA_SEQ, PATH_MFMA_SPARSE, PATH_VALU, PERIODIC, STAR, StencilError, check, lib)

SHAPES = {"star": STAR, "box": BOX}
DTYPES = {"f64": F64, "f32": F32, "bf16": BF16, "f16": F16, "bf16x3": F32_BF16X3}
BOUNDARIES = {"dirichlet": DIRICHLET, "periodic": PERIODIC}
PATHS = {"auto": PATH_AUTO, "valu": PATH_VALU, "mfma": PATH_MFMA, "mfma_sparse": PATH_MFMA_SPARSE,
         "mfma_seq": PATH_MFMA_SEQ}
PATH_NAMES = {PATH_VALU: "valu", PATH_MFMA: "mfma", PATH_MFMA_SPARSE: "mfma_sparse", PATH_MFMA_SEQ: "mfma_seq"}


def _code(table, v):
    return table[v] if isinstance(v, str) else int(v)


def torch_dtype(dtype):
    import torch
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16,
            F32_BF16X3: torch.float32}[_code(DTYPES, dtype)]


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


class Plan:
    """Owns a stencil_plan_t.  Weights are float64 in canonical order."""

    def __init__(self, shape, d, r, weights, dims, T=1, dtype="f64", boundary="dirichlet",
                 path=None, halo=None, tile_rows=None):
        w = np.ascontiguousarray(weights, dtype=np.float64)
        dims_a = (ctypes.c_int64 * len(dims))(*[int(x) for x in dims])
        h = ctypes.c_void_p()
        self._h = None
        check(lib().stencil_plan(ctypes.byref(h), _code(SHAPES, shape), int(d), int(r),
                                 w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), dims_a,
                                 int(T), _code(DTYPES, dtype), _code(BOUNDARIES, boundary)),
              "stencil_plan")
        self._h = h
        self.dims = tuple(int(x) for x in dims)
        self.dtype = _code(DTYPES, dtype)
        if path is not None:
            self.set(_abi.OPT_PATH, _code(PATHS, path))
        if halo is not None:
            self.set(_abi.OPT_HALO_VALUE, float(halo))
        if tile_rows is not None:
            self.set(_abi.OPT_TILE_ROWS, int(tile_rows))

    @property
    def handle(self):
        return self._h

    def set(self, option, value):
        check(lib().stencil_plan_set(self._h, int(option), float(value)), "stencil_plan_set")

    def info(self) -> dict:
        i = _abi.PlanInfo()
        check(lib().stencil_plan_info(self._h, ctypes.byref(i)), "stencil_plan_info")
        out = {f: getattr(i, f) for f, _ in _abi.PlanInfo._fields_}
        out["dims"] = tuple(i.dims[:i.d])
        out["path_name"] = PATH_NAMES.get(i.path, "?")
        return out

    def _check_tensor(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA (HIP) tensor")
        if tuple(t.shape) != self.dims or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.dims}")
        if t.dtype != torch_dtype(self.dtype):
            raise ValueError(f"{name} must have dtype {torch_dtype(self.dtype)}")

    def run(self, inp, out, steps, stream=None):
        self._check_tensor(inp, "in")
        self._check_tensor(out, "out")
        check(lib().stencil_run(self._h, ctypes.c_void_p(inp.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), int(steps),
                                _stream_handle(stream)), "stencil_run")
        return out

    def run_noalloc(self, inp, out, steps, stream=None):
        """stencil_run_noalloc: as run(), with the intermediate grid in the
        library's static device array (no device allocation)."""
        self._check_tensor(inp, "in")
        self._check_tensor(out, "out")
        check(lib().stencil_run_noalloc(self._h, ctypes.c_void_p(inp.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), int(steps),
                                        _stream_handle(stream)), "stencil_run_noalloc")
        return out

    def autotune(self, inp, out, steps, max_candidates=4, stream=None) -> float:
        """Choose path, T and tile rows by timing model-ranked candidates on
        inp -> out (out is overwritten).  Returns the measured GStencil/s."""
        self._check_tensor(inp, "in")
        self._check_tensor(out, "out")
        g = ctypes.c_double()
        check(lib().stencil_plan_autotune(self._h, ctypes.c_void_p(inp.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), int(steps),
                                          int(max_candidates), _stream_handle(stream),
                                          ctypes.byref(g)), "stencil_plan_autotune")
        return g.value

    def close(self):
        if self._h is not None and self._h.value:
            lib().stencil_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_batch(plans, ins, outs, steps, stream=None):
    n = len(plans)
    for p, a, b in zip(plans, ins, outs):
        p._check_tensor(a, "in")
        p._check_tensor(b, "out")
    P = (ctypes.c_void_p * n)(*[p.handle.value for p in plans])
    I = (ctypes.c_void_p * n)(*[t.data_ptr() for t in ins])
    O = (ctypes.c_void_p * n)(*[t.data_ptr() for t in outs])
    S = (ctypes.c_int64 * n)(*[int(s) for s in steps])
    check(lib().stencil_run_batch(n, P, I, O, S, _stream_handle(stream)), "stencil_run_batch")


def compose(shape, d, r, weights, T):
    """Dense (2rT+1)^d composite kernel of T steps and its support size."""
    w = np.ascontiguousarray(weights, dtype=np.float64)
    R = int(r) * int(T)
    out = np.zeros((2 * R + 1,) * int(d), dtype=np.float64)
    kt = ctypes.c_int()
    check(lib().stencil_compose(_code(SHAPES, shape), int(d), int(r),
                                w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(T),
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                ctypes.byref(kt)), "stencil_compose")
    return out, kt.value


def hw_default(dtype) -> dict:
    h = _abi.HW()
    check(lib().stencil_hw_default(_code(DTYPES, dtype), ctypes.byref(h)), "stencil_hw_default")
    return {f: getattr(h, f) for f, _ in _abi.HW._fields_}


def model_predict(shape, d, r, T, dtype, S=0.0, alpha=0.0, sparse=False, hw=None) -> dict:
    mi = _abi.ModelIn(_code(SHAPES, shape), int(d), int(r), int(T), _code(DTYPES, dtype),
                      float(S), float(alpha), int(bool(sparse)))
    mo = _abi.ModelOut()
    hwp = None
    if hw is not None:
        hwp = ctypes.byref(_abi.HW(hw["BB"], hw["PP_valu"], hw["PP_mfma"],
                                   hw.get("PP_mfma_sparse", hw["PP_mfma"])))
    check(lib().stencil_model_predict(ctypes.byref(mi), hwp, ctypes.byref(mo)),
          "stencil_model_predict")
    return {f: getattr(mo, f) for f, _ in _abi.ModelOut._fields_}


def microbench(kind: str, nbytes: int = 1 << 30) -> float:
    """Measured ceiling: 'copy' (bytes/s), 'fma_f64', 'fma_f32', 'mfma_f64',
    'mfma_f32', 'mfma_bf16', 'fma_f32_sgpr' / 'fma_f32_vgpr' (FP32 FMAs with a
    scalar-register multiplier / vector operands only) (flop/s)."""
    import torch

    kinds = ["copy", "fma_f64", "fma_f32", "mfma_f64", "mfma_f32", "mfma_bf16", "fma_f32_sgpr", "fma_f32_vgpr"]
    k = kinds.index(kind)
    buf = torch.empty(nbytes if k == 0 else 32, dtype=torch.uint8, device="cuda")
    out = ctypes.c_double()
    check(lib().stencil_microbench(k, ctypes.c_void_p(buf.data_ptr()), int(buf.numel()),
                                   _stream_handle(None), ctypes.byref(out)), "stencil_microbench")
    return out.value


def kernel_available(path, dtype, shape, d, r, T) -> bool:
    """True when a kernel fuses T steps of (shape, d, r) on `path` for dtype."""
    return bool(lib().stencil_kernel_available(_code(PATHS, path), _code(DTYPES, dtype),
                                               _code(SHAPES, shape), int(d), int(r), int(T)))


def mfma_sparsity(shape, d, r, T, dtype) -> float:
    return float(lib().stencil_mfma_sparsity(_code(SHAPES, shape), int(d), int(r), int(T),
                                             _code(DTYPES, dtype)))
