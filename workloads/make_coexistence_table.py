"""Write coexistence_pr.json: Maxwell coexistence densities of the
Peng-Robinson fluid of Sec. 4 (a = 3/49, b = 2/21, R = 1, omega = 0.344) on
T/Tc = 0.700, 0.701, ..., 0.995.  Calls only the oracle's equal-area solver.

Usage: python workloads/make_coexistence_table.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import lbm_oracle as O  # noqa: E402


def main():
    p = O.Params(1, 1, 1)
    Tc = O.critical_temperature(p)
    rows = []
    for k in range(0, 296):
        t = round(0.700 + 0.001 * k, 3)
        rv, rl, ps = O.maxwell_coexistence(t * Tc, p)
        rows.append([t, rv, rl, ps])
    out = dict(a=p.a, b=p.b, R=p.R, omega=p.omega, Tc=Tc,
               columns=["T_over_Tc", "rho_v", "rho_l", "p_sat"], rows=rows)
    with open(os.path.join(HERE, "coexistence_pr.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
