"""Writes tests/golden/slab_coexistence.json: the converged bulk densities of
a flat liquid slab under the method at T = 0.86 Tc with T held fixed (very
large c_v), computed by the FP64 oracle only (128 x 1 x 1 periodic column,
40000 steps, velocity below 1e-11 at the end).

Run from the repository root: python tests/golden/make_slab_coexistence.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lbm_oracle as O  # noqa: E402
from workloads import synth  # noqa: E402


def main():
    w = synth.slab(nx=128, ny=1, nz=1, width=64.0)
    p = O.Params(128, 1, 1, cv=1e6)
    f, g = O.init_populations(w["rho0"], w["T0"], p)
    f, g = O.run(f, g, p, 40000)
    rho, u, _ = O.fields(f, g, p)
    out = {
        "what": "converged flat-interface bulk densities of the method (oracle), T = 0.86 Tc fixed",
        "grid": [128, 1, 1], "slab_width": 64.0, "interface_width": 5.0, "steps": 40000, "cv": 1e6,
        "rho_liquid": float(rho[0, 0, 64]), "rho_vapour": float(rho[0, 0, 0]),
        "max_abs_u": float(np.max(np.abs(u))),
        "maxwell_rho_liquid": w["rho_l"], "maxwell_rho_vapour": w["rho_v"],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "slab_coexistence.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(out)


if __name__ == "__main__":
    main()
