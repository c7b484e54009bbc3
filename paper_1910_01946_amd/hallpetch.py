"""Hall-Petch analysis of a grain-size sweep (Section 3, eqs. 19-21): post-processing of the
macroscopic curves that the library computes, outside the homogenization path.

For each material, RVEs of mean grain sizes D with the GND term (c_gnd = 1) and one twin
without it (c_gnd = 0: no length scale, the paper's "infinite" grain size, flow stress
sigma_inf) run through the same load path in one handle.  At a given applied strain the
grain-boundary strengthening sigma_y / sigma_inf - 1 is fitted, in logarithms, to
C (D sqrt(rho_i))^-x (eq. 21) by least squares over the sizes; the paper reports x between
0.69 (Al) and 0.74 (Ag) at 1 % and between 0.59 (Al) and 0.73 (Ag) at 5 %.

Usage (GPU): python -m paper_1910_01946_amd.hallpetch [--n 32] [--grains 100] [--out file.json]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np


def flow_stress(strains, sigma, eps):
    """Stress at applied strain eps, linear interpolation along the curve."""
    return float(np.interp(eps, np.asarray(strains), np.asarray(sigma)))


def fit_size_effect(D, sigma_y, sigma_inf, rho_i):
    """Least-squares fit of log(sigma_y / sigma_inf - 1) = log C - x log(D sqrt(rho_i)) (eq. 21).
    Returns (C, x); needs at least two sizes with sigma_y > sigma_inf."""
    D = np.asarray(D, dtype=np.float64)
    y = np.asarray(sigma_y, dtype=np.float64) / float(sigma_inf) - 1.0
    if np.any(y <= 0) or D.size < 2:
        raise ValueError("the strengthening must be positive at two sizes at least")
    X = np.log(D * math.sqrt(rho_i))
    A = np.stack([np.ones_like(X), -X], axis=1)
    (logC, x), *_ = np.linalg.lstsq(A, np.log(y), rcond=None)
    return float(math.exp(logC)), float(x)


def run_sweep(rves, path, labels, precision=None, strains=(0.01, 0.05), rho_i=1.2e12, log=print):
    """Run the sweep through the library (one handle, all RVEs concurrently) and fit eq. 21 per
    material at each strain in strains.  Returns a dict of the curves and fits."""
    import paper_1910_01946_amd as lib

    prec = lib.RVE_MIXED if precision is None else precision
    # time-step cut-back: at 0.1 % strain per increment the twins without the GND term (the
    # lowest critical stresses) can take load steps that the local solve does not survive
    h = lib.Homogenizer(rves, precision=prec, newton_tol=1e-6, cg_tol=1e-3, max_cg=3000, max_newton=150,
                        use_graph=1, autotune=1, max_cutbacks=6)
    eps = [float(path.F_bar[k][0] - 1.0) for k in range(path.n_inc + 1)]
    curves = [[0.0] for _ in rves]
    t0 = time.perf_counter()
    for k in range(1, path.n_inc + 1):
        st = h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        for i in range(len(rves)):
            curves[i].append(float(h.macro(i)[2][0]))   # Cauchy sigma_11
        cuts = [i for i, s in enumerate(st) if s["cutbacks"]]
        log(f"increment {k} done ({time.perf_counter() - t0:.1f} s)" + (f", cut back: RVEs {cuts}" if cuts else ""))
    h.close()
    out = {"strain": eps, "labels": [[m, d] for m, d in labels], "sigma_11": curves, "fits": {}}
    for m in sorted({m for m, _ in labels}):
        idx = [i for i, (mm, d) in enumerate(labels) if mm == m and d is not None]
        twin = next(i for i, (mm, d) in enumerate(labels) if mm == m and d is None)
        for e in strains:
            if e > eps[-1] + 1e-12:
                continue
            s_inf = flow_stress(eps, curves[twin], e)
            s_y = [flow_stress(eps, curves[i], e) for i in idx]
            D = [labels[i][1] for i in idx]
            C, x = fit_size_effect(D, s_y, s_inf, rho_i)
            out["fits"][f"{m}@{e:g}"] = {"C": C, "x": x, "sigma_inf": s_inf, "sigma_y": s_y, "D": D,
                                         "strengthening": [sy / s_inf - 1.0 for sy in s_y]}
            log(f"{m} at {100 * e:g} %: x = {x:.3f}, C = {C:.3g}, sigma_inf = {s_inf / 1e6:.2f} MPa, "
                f"strengthening {[round(sy / s_inf - 1.0, 4) for sy in s_y]}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--grains", type=int, default=100)
    ap.add_argument("--increments", type=int, default=50)
    ap.add_argument("--strain", type=float, default=0.05)
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch  # noqa: F401

    import synth

    rves, path, labels = synth.hall_petch_workload(n=args.n, n_grains=args.grains, strain_max=args.strain,
                                                   n_inc=args.increments)
    res = run_sweep(rves, path, labels, log=lambda s: print(s, file=sys.stderr, flush=True))
    res["config"] = {"n": args.n, "grains": args.grains, "increments": args.increments, "strain": args.strain}
    text = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(json.dumps({k: {kk: v[kk] for kk in ("x", "C")} for k, v in res["fits"].items()}))


if __name__ == "__main__":
    main()
