"""ctypes declarations of the C ABI in include/stencil.h.

Argument marshalling only: every step of a sweep runs in the HIP library.
Loading fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstencil_mi355.so")

STAR, BOX = 0, 1
F64, F32, BF16, F16, F32_BF16X3 = 0, 1, 2, 3, 4
DIRICHLET, PERIODIC = 0, 1
PATH_AUTO, PATH_VALU, PATH_MFMA, PATH_MFMA_SPARSE, PATH_MFMA_SEQ = 0, 1, 2, 3, 4
OPT_PATH, OPT_HALO_VALUE, OPT_TILE_ROWS, OPT_T = 1, 2, 3, 4
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "ALIAS", 4: "OOM", 5: "HIP"}

SYMBOLS = ["stencil_plan", "stencil_plan_set", "stencil_plan_info", "stencil_run",
           "stencil_run_batch", "stencil_plan_destroy", "stencil_last_error", "stencil_compose",
           "stencil_hw_default", "stencil_model_predict", "stencil_mfma_sparsity",
           "stencil_plan_autotune", "stencil_microbench", "stencil_kernel_available",
           "stencil_run_noalloc"]
NOALLOC_SCRATCH_BYTES = 64 << 20  # STENCIL_NOALLOC_SCRATCH_BYTES


class PlanInfo(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int), ("d", ctypes.c_int), ("r", ctypes.c_int),
                ("T", ctypes.c_int), ("dtype", ctypes.c_int), ("boundary", ctypes.c_int),
                ("path", ctypes.c_int), ("dims", ctypes.c_int64 * 3), ("K", ctypes.c_int),
                ("K_T", ctypes.c_int), ("alpha", ctypes.c_double), ("S", ctypes.c_double),
                ("gamma", ctypes.c_double), ("halo", ctypes.c_double),
                ("workspace_bytes", ctypes.c_int64), ("predicted_gst_valu", ctypes.c_double),
                ("predicted_gst_mfma", ctypes.c_double), ("predicted_winner", ctypes.c_int),
                ("scenario", ctypes.c_int), ("tile_rows", ctypes.c_int), ("T_fused", ctypes.c_int)]


class HW(ctypes.Structure):
    _fields_ = [("BB", ctypes.c_double), ("PP_valu", ctypes.c_double),
                ("PP_mfma", ctypes.c_double), ("PP_mfma_sparse", ctypes.c_double)]


class ModelIn(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int), ("d", ctypes.c_int), ("r", ctypes.c_int),
                ("T", ctypes.c_int), ("dtype", ctypes.c_int), ("S", ctypes.c_double),
                ("alpha", ctypes.c_double), ("sparse", ctypes.c_int)]


class ModelOut(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int), ("K_T", ctypes.c_int), ("D", ctypes.c_double),
                ("alpha", ctypes.c_double), ("S", ctypes.c_double), ("gamma", ctypes.c_double),
                ("C_valu", ctypes.c_double), ("C_mfma", ctypes.c_double), ("M", ctypes.c_double),
                ("I_valu", ctypes.c_double), ("I_mfma", ctypes.c_double),
                ("ridge_valu", ctypes.c_double), ("ridge_mfma", ctypes.c_double),
                ("P_valu", ctypes.c_double), ("P_mfma_raw", ctypes.c_double),
                ("P_mfma", ctypes.c_double), ("gst_valu", ctypes.c_double),
                ("gst_mfma", ctypes.c_double), ("ratio", ctypes.c_double),
                ("scenario", ctypes.c_int), ("sweet_spot", ctypes.c_int), ("winner", ctypes.c_int),
                ("halo_valu", ctypes.c_double), ("C_mfma_seq", ctypes.c_double),
                ("gst_mfma_seq", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i64p, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), \
        ctypes.POINTER(ctypes.c_double)
    L.stencil_plan.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int, ctypes.c_int, dp,
                               i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.stencil_plan_set.argtypes = [vp, ctypes.c_int, ctypes.c_double]
    L.stencil_plan_info.argtypes = [vp, ctypes.POINTER(PlanInfo)]
    L.stencil_run.argtypes = [vp, vp, vp, i64, vp]
    L.stencil_run_noalloc.argtypes = [vp, vp, vp, i64, vp]
    L.stencil_run_batch.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.POINTER(vp), i64p, vp]
    L.stencil_plan_destroy.argtypes = [vp]
    L.stencil_plan_destroy.restype = None
    L.stencil_last_error.restype = ctypes.c_char_p
    L.stencil_compose.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp,
                                  ctypes.POINTER(ctypes.c_int)]
    L.stencil_hw_default.argtypes = [ctypes.c_int, ctypes.POINTER(HW)]
    L.stencil_model_predict.argtypes = [ctypes.POINTER(ModelIn), ctypes.POINTER(HW),
                                        ctypes.POINTER(ModelOut)]
    L.stencil_plan_autotune.argtypes = [vp, vp, vp, i64, ctypes.c_int, vp, dp]
    L.stencil_microbench.argtypes = [ctypes.c_int, vp, i64, vp, dp]
    L.stencil_microbench.restype = ctypes.c_int
    L.stencil_mfma_sparsity.argtypes = [ctypes.c_int] * 5
    L.stencil_mfma_sparsity.restype = ctypes.c_double
    L.stencil_kernel_available.argtypes = [ctypes.c_int] * 6
    L.stencil_kernel_available.restype = ctypes.c_int
    for name in ("stencil_plan", "stencil_plan_set", "stencil_plan_info", "stencil_run",
                 "stencil_plan_autotune", "stencil_run_noalloc",
                 "stencil_run_batch", "stencil_compose", "stencil_hw_default",
                 "stencil_model_predict"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class StencilError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().stencil_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


def check(code: int, where: str):
    if code != 0:
        raise StencilError(code, where)
