"""Write tests/golden/c1_cu16_curve.json with the oracle only (test infrastructure).

The 16^3 FP64 workload (8 Voronoi grains, seed 101, Cu, tau0 = 10 MPa, no gradient term,
uniaxial tension to 1 % in 20 increments at 1e-3/s): <P> and <F> after every increment, the
oracle converged to |dF| <= 1e-12 (CG 1e-11).
Run from the repository root: python tests/golden/make_c1_curve.py
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import solver  # noqa: E402


def main():
    rves, path = synth.workload("cu16")
    s = solver.RVESolver(rves[0], newton_tol=1e-12, cg_tol=1e-11, max_cg=20000, max_newton=80)
    t0 = time.time()
    P, F = [], []
    for k in range(1, path.n_inc + 1):
        st = s.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        if not st["converged"]:
            raise RuntimeError(f"increment {k}: {st}")
        Pa, Fa, _ = s.macro()
        P.append(Pa.tolist())
        F.append(Fa.tolist())
        print(f"increment {k}: <P>_11 {Pa[0]:.12e} newton {st['newton']} cg {st['cg']} ({time.time() - t0:.0f} s)",
              flush=True)
    out = os.path.join(ROOT, "tests", "golden", "c1_cu16_curve.json")
    with open(out, "w") as f:
        json.dump({"workload": "cu16 (16^3, 8 grains, Cu, tau0 10 MPa, c_gnd 0), 20 increments to 1 %",
                   "newton_tol": 1e-12, "cg_tol": 1e-11, "P_avg": P, "F_avg": F,
                   "script": "tests/golden/make_c1_curve.py (calls oracle/ only)"}, f, indent=1)
    print("wrote", out)


if __name__ == "__main__":
    main()
