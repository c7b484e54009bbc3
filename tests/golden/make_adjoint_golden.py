"""Write tests/golden/adjoint_cu64g100_8cubed.json with the oracle only (test infrastructure).

The adjoint workload (100 grains, Cu, c_gnd = 1) on an 8^3 grid, first 6 increments of its
load path, FP64 oracle converged to |dF| <= 1e-14 (CG 1e-13):
  * curve: <P>_11 at each increment at theta = (tau0, K, y_c, c_gnd);
  * dcurve: d<P>_11,k / d theta_j by central differences of the whole oracle run, relative
    steps 1e-6 and 4e-6 (their difference estimates the quotient's error);
  * target: the curve at theta* = (1.1 tau0, 0.9 K, 1.1 y_c, 1.2 c_gnd) plus Gaussian noise of
    0.5 % of its largest stress (seed 205), the synthetic target of the curve loss
    L = sum_k (<P>_11,k - target_k)^2.
Run from the repository root: python tests/golden/make_adjoint_golden.py
"""
from __future__ import annotations

import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import solver  # noqa: E402

N, N_INC = 8, 6
TOL = dict(newton_tol=1e-14, cg_tol=1e-13, max_cg=20000, max_newton=80)


def curve(rve, path, theta):
    r = dataclasses.replace(rve, material=synth.with_params(rve.material, theta))
    s = solver.RVESolver(r, **TOL)
    out = []
    for k in range(1, path.n_inc + 1):
        st = s.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        if not st["converged"]:
            raise RuntimeError(f"increment {k} did not converge: {st}")
        out.append(float(s.macro()[0][0]))
    return np.array(out)


def main():
    rve, path, theta = synth.adjoint_workload(n_override=N, n_inc_override=N_INC)
    t0 = time.time()
    base = curve(rve, path, theta)
    print(f"base curve {base} ({time.time() - t0:.0f} s)", flush=True)
    dcurve = {}
    for rel in (1e-6, 4e-6):
        d = np.zeros((N_INC, 4))
        for j in range(4):
            h = rel * theta[j]
            tp = list(theta)
            tm = list(theta)
            tp[j] += h
            tm[j] -= h
            d[:, j] = (curve(rve, path, tp) - curve(rve, path, tm)) / (2 * h)
            print(f"rel step {rel:g}, parameter {synth.ADJOINT_PARAMS[j]}: {d[:, j]}", flush=True)
        dcurve[str(rel)] = d.tolist()
    star = (1.1 * theta[0], 0.9 * theta[1], 1.1 * theta[2], 1.2 * theta[3])
    cs = curve(rve, path, star)
    target = cs + 0.005 * np.abs(cs).max() * synth.gaussian_noise(205, N_INC)
    rec = {"workload": "adjoint workload (cu64g100 grains) at 8^3, increments 1-6", "n": N, "n_inc": N_INC,
           "params": list(synth.ADJOINT_PARAMS), "theta": list(theta), "theta_star": list(star),
           "tolerances": TOL, "curve": base.tolist(), "dcurve_dtheta": dcurve, "target": target.tolist(),
           "script": "tests/golden/make_adjoint_golden.py (calls oracle/ only)"}
    out = os.path.join(ROOT, "tests", "golden", "adjoint_cu64g100_8cubed.json")
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {out} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
