"""Oracle for the stencil sweep: test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the GPU library
(``paper_2603_00477_amd``) and does not import it.

Contents
--------
core     FP64 stencil sweep (plain C, OpenMP) behind ctypes: full grid and
         dependency-cone windows.
brute    Independent pure-Python builder of the affine step operator for tiny
         grids (exact rationals), used to pin ``core``.
compose  T-fold composite kernel of kernel fusion and its support size.
model    The paper's roofline model, redundancy factors and scenario criteria
         as closed forms.
"""
from . import core, brute, compose, model  # noqa: F401
