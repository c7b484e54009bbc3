"""Benchmark: voxel-iterations/s of the FFT strain-gradient crystal-plasticity loop on one MI355X.

A step is one load increment of the whole workload: for every RVE, the Newton iterations
of the Galerkin-FFT equilibrium solve (constitutive updates, projected residuals and
conjugate-gradient matvecs), the commit, and the Fourier-space Nye tensor and GND
densities.  A voxel-iteration is one voxel through one projected-operator application
(a Newton residual or a CG matvec).  Inputs are seeded synthetic RVEs resident on the
GPU before the timed region; rve_create is outside it.

The default workload is the 64^3 strain-gradient RVE (64 Voronoi grains, Cu, 5 % tension
in 50 increments) in the mixed-precision form; the same increments are then timed in the
plain FP64 form, and the macroscopic stress of the two is compared.  The roofline object
reports the kernel family with the largest share of the timed increments, timed with
events that the kernel dispatches record on the RVE's stream, in replays of the timed
increments from the same saved state; the headline value comes from the uninstrumented
pass.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cu64|cu16|al128|sweep32|cu64g100]
                       [--precision mixed|fp64] [--no-fp64-compare] [--no-cpu-baseline]
                       [--no-roofline] [--roofline-kernel auto|mid|cg_prep|plane_fwd|...]
       python bench.py --copy-calibration   (plain device copy of known size, for the
                                             FETCH_SIZE / WRITE_SIZE counter scale)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "voxel-iterations/s per MI355X, mixed-prec+batched vs plain FP64 at 1e-4"

# kernel families of the timing interface: kernel names (as profilers list them) and the
# source files whose change invalidates stored counter readings
_CONST_SRC = ["constitutive.hip", "kernels.h", "timing.h", "common.h"]
_PLANE_SRC = ["plane.hip", "spectral.h", "fft.h", "kernels.h", "timing.h", "common.h"]
_MID_SRC = ["spectral.hip", "spectral.h", "fft.h", "kernels.h", "timing.h", "common.h"]
FAMILY_KERNELS = {
    "slip_fast": ("k_slip_fast", _CONST_SRC),
    "slip_slow": ("k_slip_slow", _CONST_SRC),
    "stress_tangent": ("k_stress_tangent", _CONST_SRC),
    "cg_prep": ("k_cg_prep", _PLANE_SRC),
    "plane_fwd": ("k_plane_fwd", _PLANE_SRC),
    "mid": ("k_mid", _MID_SRC),
    "plane_inv": ("k_plane_inv", _PLANE_SRC),
}
SPECTRAL = ("cg_prep", "plane_fwd", "mid", "plane_inv")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="cu64")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--newton-tol", type=float, default=1e-6)
    ap.add_argument("--cg-tol", type=float, default=1e-3)
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--roofline-kernel", default="auto", choices=["auto"] + list(FAMILY_KERNELS),
                    help="kernel family of the roofline object (auto: the largest share of the timed "
                         "increments)")
    ap.add_argument("--rves", type=int, default=None, help="use only the first R RVEs of the workload")
    ap.add_argument("--copy-calibration", action="store_true")
    return ap.parse_args()


# (warmup, timed) increments per workload
DEFAULTS = {"cu16": (2, 10), "cu64": (3, 8), "al128": (2, 3), "sweep32": (2, 3), "cu64g100": (3, 8)}


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


def source_digest(files):
    """Digest of the code of the given sources, comments and blank lines left out (a change
    of wording does not invalidate stored counter readings; a change of code does)."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1910_01946_amd", "csrc", f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(code.encode("utf-8"))
    return h.hexdigest()[:16]


def stored_traffic(family: str, workload: str, precision: str):
    """HBM bytes per launch from the committed counter summary of this kernel and workload
    (FETCH_SIZE and WRITE_SIZE, each scaled by the reading of a plain copy); None when the
    summary is missing or the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_{family}_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^traffic_bytes_per_launch\s*=\s*([0-9.eE+]+)", text, re.M)
    d = re.search(r"^source_digest\s*=\s*([0-9a-f]+)", text, re.M)
    if not m or not d or d.group(1) != source_digest(FAMILY_KERNELS[family][1]):
        return None
    return float(m.group(1))


def _timed(h, path, W, K, tag):
    import torch

    vi = 0.0
    it_stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(W + 1, W + K + 1):
        st = h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        vi += sum(s["voxel_iterations"] for s in st)
        it_stats.append((sum(s["newton_iters"] for s in st), sum(s["cg_iters"] for s in st),
                         sum(s["fp64_fallback"] for s in st)))
        print(f"[{tag}] timed increment {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return vi, time.perf_counter() - t0, it_stats


def run_leg(lib, rves, path, prec, W, K, args, roof_family=None):
    """Warm up W increments, then time K increments without instrumentation.  With
    roof_family, the committed state after the warmup is restored and the same K
    increments are replayed: once with kernel-timing events on every family (the share
    of each; "auto" then picks the largest), once with events on the chosen family only
    (its live average launch duration)."""
    h = lib.Homogenizer(rves, precision=prec, newton_tol=args.newton_tol, cg_tol=args.cg_tol, max_cg=3000,
                        max_newton=150)
    tag = "mixed" if prec == lib.RVE_MIXED else "fp64"
    for k in range(1, W + 1):
        h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        print(f"[{tag}] warmup increment {k} done", file=sys.stderr, flush=True)
    saved = h.save_state() if roof_family else None
    vi, T, it_stats = _timed(h, path, W, K, tag)
    P = [h.macro(i)[0] for i in range(len(rves))]
    out = {"value": vi / T, "T": T, "vi": vi, "iters": it_stats, "P": P}
    if roof_family:
        h.load_state(saved)
        h.timing_start(list(FAMILY_KERNELS))
        _, T2, _ = _timed(h, path, W, K, tag + " replay, events on all families")
        out["share"] = {f: h.timing_read(f)[1] / (1e3 * T2) for f in FAMILY_KERNELS}
        if roof_family == "auto":
            roof_family = max(out["share"], key=out["share"].get)
        h.load_state(saved)
        h.timing_start([roof_family])
        _, T1, it1 = _timed(h, path, W, K, tag + " replay, events on " + roof_family)
        out["roof"] = (roof_family, h.timing_read(roof_family), T1, it1 == it_stats)
        h.timing_start(())
    h.close()
    return out


def roofline(leg, workload, precision):
    """Roofline object of the family timed in the replay (HBM bound for the spectral
    kernels: algorithmic bytes per launch over the event-measured average duration)."""
    fam, (n, ms, units), T1, same = leg["roof"]
    if n == 0:
        return None
    out = {"kernel": FAMILY_KERNELS[fam][0], "launches": n, "avg_launch_us": 1e3 * ms / n,
           "replay_matches_timed_iterations": same,
           "share_of_replay_with_events_on_all_families": {f: round(v, 4) for f, v in leg["share"].items()}}
    if fam in SPECTRAL:
        achieved = units / (ms * 1e-3) / 1e9
        traffic = stored_traffic(fam, workload, precision)
        out.update({"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": units / n,
                    "traffic": traffic})
    else:
        # the local Newton solves have a data-dependent iteration count; no algorithmic
        # operation count per launch is defined for them
        out.update({"bound": "alu", "achieved": None, "peak": 78.6, "unit": "TFLOP/s", "frac": None,
                    "traffic": None})
    return out


def copy_calibration():
    """A plain device copy of 1 GiB, five times: the reference for scaling the FETCH_SIZE and
    WRITE_SIZE counters (each copy reads and writes exactly 2^30 bytes)."""
    import torch

    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 5}))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch  # noqa: F401  (before the library: one HIP runtime in the process)

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
    roof_family = None if args.no_roofline else args.roofline_kernel
    main_leg = run_leg(lib, rves, path, prec, W, K, args, roof_family)
    nvox = sum(r.n_vox for r in rves)
    config = {"workload": args.workload, "n_rve": len(rves), "voxels": nvox,
              "grids": sorted({tuple(r.n) for r in rves}), "increments_timed": [W + 1, W + K],
              "newton_tol": args.newton_tol, "cg_tol": args.cg_tol, "precision": args.precision,
              "newton_cg_fallback_per_increment": main_leg["iters"], "P11_last": float(main_leg["P"][0][0])}
    if prec == lib.RVE_MIXED and not args.no_fp64_compare:
        ref = run_leg(lib, rves, path, lib.RVE_FP64, W, K, args)
        per_rve = [abs(a[0] - b[0]) / abs(b[0]) for a, b in zip(main_leg["P"], ref["P"])]
        rel = max(per_rve)
        config["fp64_form"] = {"value": ref["value"], "ms_per_step": 1e3 * ref["T"] / K,
                               "newton_cg_fallback_per_increment": ref["iters"],
                               "speedup_mixed_over_fp64": main_leg["value"] / ref["value"],
                               "P11_rel_diff_mixed_vs_fp64": rel}
        if len(per_rve) > 1:
            config["fp64_form"]["P11_rel_diff_per_rve"] = [float("%.3g" % v) for v in per_rve]
    line = {
        "metric": METRIC,
        "value": main_leg["value"],
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * main_leg["T"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == lib.RVE_MIXED else "f64",
        "data": "synthetic",
        "config": config,
    }
    if roof_family:
        line["roofline"] = roofline(main_leg, args.workload, args.precision)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
