"""Benchmark: voxel-iterations/s of the FFT strain-gradient crystal-plasticity loop on one MI355X.

A step is one load increment of the whole workload: for every RVE, the Newton iterations
of the Galerkin-FFT equilibrium solve (constitutive updates, projected residuals and
conjugate-gradient matvecs), the commit, and the Fourier-space Nye tensor and GND
densities.  A voxel-iteration is one voxel through one projected-operator application
(a Newton residual or a CG matvec).  Inputs are seeded synthetic RVEs resident on the
GPU before the timed region; rve_create is outside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c2|c3|c1]
                       [--precision mixed|fp64] [--no-cpu-baseline] [--no-roofline]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--newton-tol", type=float, default=1e-6)
    ap.add_argument("--cg-tol", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--rves", type=int, default=None, help="use only the first R RVEs of the workload")
    return ap.parse_args()


DEFAULTS = {"c1": (2, 10), "c2": (3, 8), "c3": (2, 3), "c4": (2, 3), "c5": (3, 8)}


def cpu_baseline(workload: str):
    """Time the CPU oracle, single-threaded, on a bounded sample: the first increment of the
    workload's first RVE regridded to 8^3 (same seed, grains, material and load path)."""
    code = r"""
import json, sys, time
sys.path.insert(0, %r)
import synth
from oracle import solver
rves, path = synth.workload(%r, n_override=8)
r = rves[0]
s = solver.RVESolver(r, newton_tol=1e-8, cg_tol=1e-6)
t = time.perf_counter()
st = s.step(path.F_bar[1], path.mask, path.P_bar[1], path.dt)
dt = time.perf_counter() - t
print(json.dumps({"vi": st["voxel_iterations"], "sec": dt, "conv": st["converged"]}))
""" % (ROOT, workload)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=900)
    rec = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": rec["vi"] / rec["sec"], "unit": "voxel-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"increment 1 of workload {workload} RVE 0 regridded to 8^3 "
                      f"({rec['vi']:.0f} voxel-iterations in {rec['sec']:.1f} s, FP64 numpy, 1 thread)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import synth
    import paper_1910_01946_amd as lib

    lib.lib()
    rves, path = synth.workload(args.workload)
    if args.rves:
        rves = rves[: args.rves]
    w_def, k_def = DEFAULTS.get(args.workload, (2, 5))
    W = args.warmup if args.warmup is not None else w_def
    K = args.steps if args.steps is not None else k_def
    K = max(1, min(K, path.n_inc - W))
    prec = lib.RVE_MIXED if args.precision == "mixed" else lib.RVE_FP64
    h = lib.Homogenizer(rves, precision=prec, newton_tol=args.newton_tol, cg_tol=args.cg_tol, max_cg=3000,
                        max_newton=150)
    for k in range(1, W + 1):
        h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        print(f"warmup increment {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    vi = 0.0
    it_stats = []
    t0 = time.perf_counter()
    for k in range(W + 1, W + K + 1):
        st = h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        vi += sum(s["voxel_iterations"] for s in st)
        it_stats.append((sum(s["newton_iters"] for s in st), sum(s["cg_iters"] for s in st), sum(s["fp64_fallback"] for s in st)))
        print(f"timed increment {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    P, F, sig = h.macro(0)
    nvox = sum(r.n_vox for r in rves)
    line = {
        "metric": "voxel-iterations/s per MI355X, mixed-prec+batched vs plain FP64 at 1e-4",
        "value": vi / T,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * T / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 spectral / f64 constitutive" if prec == lib.RVE_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "n_rve": len(rves), "voxels": nvox,
                   "grids": sorted({tuple(r.n) for r in rves}), "increments_timed": [W + 1, W + K],
                   "newton_tol": args.newton_tol, "cg_tol": args.cg_tol,
                   "newton_cg_iterations": it_stats, "P11_last": float(P[0])},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
