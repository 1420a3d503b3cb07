"""Write precision_windows_16384.json: FP64 oracle values of the 16384^2
Box-2D2R precision workload after 1000 steps on a sampled window.

The workload: periodic 16384 x 16384 grid, u0 = sin(2 pi x) sin(2 pi y) +
1e-3 U[0,1) (stencil_inputs.smooth_grid, data seed 4000), 25 weights U[0,1)
normalised to sum 1 (weight seed 4500), 1000 explicit steps.  The window is
evaluated by oracle.core.run_window (the dependency cone of the window only,
bit-identical to the full-grid oracle) for four inputs: the float64 data
(end-to-end error of every mode) and the data rounded to bf16, f16 and
float32 storage (arithmetic error of the bf16, f16 and compensated bf16x3
modes), always with the float64 weights.

Calls only stencil_inputs and oracle/.  Run from the repository root:
    python tests/golden/make_precision_windows.py
(about 5 minutes per input on 8 host cores).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import stencil_inputs as si  # noqa: E402
from oracle import core  # noqa: E402

N = 16384
STEPS = 1000
LO = (5000, 12000)
HI = (5008, 12008)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_windows_16384.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha1(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def main():
    u0 = si.smooth_grid((N, N), seed=si.data_seed(4, 0))
    w = si.normalised_weights(25, seed=si.weight_seed(4, 0))
    out = dict(_source=("FP64 oracle (oracle.core.run_window), written by "
                        "tests/golden/make_precision_windows.py"),
               pattern="box", d=2, r=2, dims=[N, N], boundary="periodic", steps=STEPS,
               data_seed=si.data_seed(4, 0), weight_seed=si.weight_seed(4, 0),
               weights=[float(x) for x in w], u0_sha1=digest(u0), lo=list(LO), hi=list(HI),
               windows={})
    for name in ("f64", "bf16", "f16", "f32"):
        src = u0 if name == "f64" else si.round_to(u0, name)[0]
        t0 = time.time()
        win = core.run_window("box", 2, 2, w, src, STEPS, LO, HI, "periodic")
        out["windows"][name] = dict(input_sha1=digest(src), max_abs_input=float(np.max(np.abs(src))),
                                    values=[[float(v) for v in row] for row in win])
        print(f"{name}: {time.time() - t0:.0f} s", flush=True)
        del src
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
