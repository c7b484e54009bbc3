"""Benchmark: voxel-iterations/s of the FFT strain-gradient crystal-plasticity loop on one MI355X.

A step is one load increment of the whole workload: for every RVE, the Newton iterations of
the Galerkin-FFT equilibrium solve (constitutive updates, projected residuals and
conjugate-gradient matvecs), the commit, and the Fourier-space Nye tensor and GND densities.
A voxel-iteration is one voxel through one projected-operator application (a Newton residual
or a CG matvec) of the solve that produced the committed increment; applies of failed
attempts (an FP64 retry of the mixed form, a failed direct attempt before load continuation)
are reported separately and not counted.  Inputs are seeded synthetic RVEs resident on the
GPU before the timed region; rve_create is outside it.

Default workload: the grain-size sweep, 32 RVEs of uneven size (32^3 to 96^3, 16 to 128
grains, Cu / Ag / Ni, 3 % tension in 30 increments) in one handle: the batched mixed form
(FP32 spectra, FP16 tangent copy, FP64 constitutive update; CG chunks as HIP graphs; RVEs
driven concurrently, one stream each; autotuned z-pass tiles).  The W warmup increments run
once in the mixed form; from that saved state the same K increments are timed in the mixed
form and in the plain FP64 form, and the macroscopic stress of the two is compared.

The roofline object reports the kernel family with the largest share of a serialised replay
(one RVE at a time, so that kernels do not overlap) of the first R timed increments, from
events that the kernel dispatches record on the RVE's stream; the headline value comes from
the uninstrumented pass.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload sweep32|cu64|cu16|al128|cu64g100]
                       [--no-fp64-compare] [--no-cpu-baseline] [--no-roofline] [--replay R]
       python bench.py --copy-calibration   (plain device copy of known size, for the
                                             FETCH_SIZE / WRITE_SIZE counter scale)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
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
    "cg_grad": ("k_cg_grad", _PLANE_SRC),
    "plane_div": ("k_plane_fwd", _PLANE_SRC),
    "mid3": ("k_mid", _MID_SRC),
    "plane_w": ("k_plane_inv", _PLANE_SRC),
}
# the spectral families: the CG iterations (factorised projection: prep, divergence pass, z
# pass on three components, inverse pass, gradient pass) and the nine-component passes of the
# residual evaluations
SPECTRAL = ("cg_prep", "plane_div", "mid3", "plane_w", "cg_grad", "plane_fwd", "mid", "plane_inv")
# the kernel instantiation each spectral family runs in the mixed form (FP32 spectra, FP16
# tangent copy) and in the FP64 form
INSTANTIATION = {
    ("cg_prep", "mixed"): "k_cg_prep<float, K16=1, TR=0>", ("cg_prep", "fp64"): "k_cg_prep<double, 0, 0>",
    ("plane_div", "mixed"): "k_plane_fwd<float, PF_DIV, ...>", ("plane_div", "fp64"): "k_plane_fwd<double, PF_DIV, ...>",
    ("mid3", "mixed"): "k_mid<float, MID_GREEN3, ...>", ("mid3", "fp64"): "k_mid<double, MID_GREEN3, ...>",
    ("plane_w", "mixed"): "k_plane_inv<float, PI_OUT_T, ...>", ("plane_w", "fp64"): "k_plane_inv<double, PI_OUT_T, ...>",
    ("cg_grad", "mixed"): "k_cg_grad<float>", ("cg_grad", "fp64"): "k_cg_grad<double>",
    ("plane_fwd", "mixed"): "k_plane_fwd<float, PF_F64, ...>", ("plane_fwd", "fp64"): "k_plane_fwd<double, PF_F64, ...>",
    ("mid", "mixed"): "k_mid<float, MID_GREEN, ...>", ("mid", "fp64"): "k_mid<double, MID_GREEN, ...>",
    ("plane_inv", "mixed"): "k_plane_inv<float, PI_RESID, ...>", ("plane_inv", "fp64"): "k_plane_inv<double, PI_RESID, ...>",
}
NEWTON_TOL, CG_TOL = 1e-6, 1e-3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="sweep32")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="issue CG chunks kernel by kernel")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--replay", type=int, default=2, help="timed increments replayed for the roofline")
    ap.add_argument("--rves", type=int, default=None, help="use only the first R RVEs of the workload")
    ap.add_argument("--copy-calibration", action="store_true")
    return ap.parse_args()


# (warmup, timed) increments per workload when not given
DEFAULTS = {"cu16": (2, 10), "cu64": (5, 20), "al128": (2, 3), "sweep32": (5, 20), "cu64g100": (5, 20)}


def host_info():
    cpu = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            m = re.search(r"^model name\s*:\s*(.+)$", f.read(), re.M)
            cpu = m.group(1).strip() if m else cpu
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "sched_affinity": len(os.sched_getaffinity(0)), "cpu": cpu}


_ORACLE_SAMPLE = r"""
import json, sys, time
sys.path.insert(0, %r)
import synth
from oracle import solver
rves, path = synth.workload(%r, n_override=8)
r = rves[%d]
s = solver.RVESolver(r, newton_tol=%r, cg_tol=%r, max_cg=3000, max_newton=150)
vi, sec = 0.0, 0.0
for k in range(1, %d + 1):
    t = time.perf_counter()
    st = s.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
    sec += time.perf_counter() - t
    assert st["converged"], st
    vi += st["voxel_iterations"]
print(json.dumps({"vi": vi, "sec": sec}))
"""


def cpu_baseline(workload: str, n_rve: int):
    """The CPU oracle as it stands (FP64 numpy, one thread per process) at the benchmark's
    tolerances on a bounded sample of the workload: increments 1-2 of its RVEs regridded to 8^3.
    One process alone gives the single-core rate; then one process per available core (at most
    16, each on a different RVE of the workload, the RVEs being independent) gives the all-cores
    rate."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    n_inc = 2

    def run(rves):
        procs = [subprocess.Popen([sys.executable, "-c", _ORACLE_SAMPLE % (ROOT, workload, r, NEWTON_TOL, CG_TOL,
                                                                            n_inc)],
                                  stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env) for r in rves]
        t0 = time.perf_counter()
        recs = []
        for p in procs:
            out, err = p.communicate(timeout=900)
            if p.returncode != 0:
                raise RuntimeError(err[-2000:])
            recs.append(json.loads(out.strip().splitlines()[-1]))
        return recs, time.perf_counter() - t0

    one, _ = run([0])
    single = one[0]["vi"] / one[0]["sec"]
    cores = max(1, min(16, len(os.sched_getaffinity(0)), n_rve))
    many, wall = run(list(range(cores)))
    total_vi = sum(r["vi"] for r in many)
    host = host_info()
    return {"value": total_vi / wall, "unit": "voxel-iterations/s", "cores": cores, "kind": "oracle",
            "single_core_value": single,
            "sample": f"increments 1-{n_inc} of the workload's RVEs regridded to 8^3 at newton_tol {NEWTON_TOL:g}, "
                      f"cg_tol {CG_TOL:g} (FP64 numpy, one thread per process); single core: RVE 0 "
                      f"({one[0]['vi']:.0f} voxel-iterations in {one[0]['sec']:.1f} s); all cores: {cores} processes "
                      f"on RVEs 0-{cores - 1} ({total_vi:.0f} voxel-iterations in {wall:.1f} s wall)",
            "host": host}


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


def timed(h, path, first, K, tag):
    """Time increments first..first+K-1 of the load path (whole rve_step_increment calls)."""
    import torch

    vi = disc = 0.0
    per_inc, P = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(first, first + K):
        t = time.perf_counter()
        st = h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        dt = time.perf_counter() - t
        vi += sum(s["voxel_iterations"] for s in st)
        disc += sum(s["discarded_voxel_iterations"] for s in st)
        per_inc.append({"increment": k, "ms": round(1e3 * dt, 2),
                        "newton": sum(s["newton_iters"] for s in st), "cg": sum(s["cg_iters"] for s in st),
                        "fp64_fallbacks": sum(s["fp64_fallback"] for s in st),
                        "continuations": sum(1 for s in st if s["continuation_stages"])})
        P.append([h.macro(i)[0][0] for i in range(h.n_rve)])
        print(f"[{tag}] timed increment {k} done ({1e3 * dt:.0f} ms)", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return {"T": time.perf_counter() - t0, "vi": vi, "discarded_vi": disc, "per_increment": per_inc, "P11": P}


class ProfilerRegion:
    """The replay is the region a profiler run with rocprofv3 --selected-regions records:
    roctxProfilerResume(0) before it and roctxProfilerPause(0) after it (no effect without a
    profiler; skipped if the ROCm tracer library is absent)."""

    def __init__(self):
        import ctypes
        self.L = None
        for name in ("libroctx64.so", "/opt/rocm/lib/libroctx64.so"):
            try:
                self.L = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if self.L is not None:
            self.L.roctxProfilerResume.argtypes = [ctypes.c_uint64]
            self.L.roctxProfilerPause.argtypes = [ctypes.c_uint64]

    def __enter__(self):
        if self.L is not None:
            self.L.roctxProfilerResume(0)
        return self

    def __exit__(self, *exc):
        if self.L is not None:
            self.L.roctxProfilerPause(0)
        return False


def roofline_replay(lib, rves, path, state, first, R, opts):
    """Serialised replay (one host worker, so RVEs and kernels do not overlap) of R increments
    from the saved state, with kernel-timing events on every family."""
    h = lib.Homogenizer(rves, precision=lib.RVE_MIXED, **dict(opts, workers=1, use_graph=0))
    h.load_state(state)
    h.timing_start(list(FAMILY_KERNELS))
    t0 = time.perf_counter()
    with ProfilerRegion():
        for k in range(first, first + R):
            h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
            print(f"[serialised replay with events] increment {k} done", file=sys.stderr, flush=True)
    T = time.perf_counter() - t0
    fam = {f: h.timing_read(f) for f in FAMILY_KERNELS}
    h.timing_start(())
    h.close()
    return fam, T


def roofline(fam, T, workload):
    share = {f: ms / (1e3 * T) for f, (n, ms, u) in fam.items()}
    per = []
    for f in SPECTRAL:
        n, ms, units = fam[f]
        if n == 0:
            continue
        achieved = units / (ms * 1e-3) / 1e9
        per.append({"family": f, "kernel": FAMILY_KERNELS[f][0], "instantiation": INSTANTIATION[(f, "mixed")],
                    "launches": n,
                    "avg_launch_us": 1e3 * ms / n, "algorithmic_bytes_per_launch": units / n,
                    "achieved": achieved, "frac": achieved / HBM_PEAK_GBS, "share": round(share[f], 4),
                    "traffic": stored_traffic(f, workload, "mixed")})
    dom = max(share, key=share.get)
    out = {"kernel": FAMILY_KERNELS[dom][0], "family": dom,
           "share_of_serialised_replay": {f: round(v, 4) for f, v in share.items()}}
    if dom in SPECTRAL:
        d = next(p for p in per if p["family"] == dom)
        out.update({"instantiation": d["instantiation"], "bound": "hbm", "achieved": d["achieved"],
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d["frac"], "traffic": d["traffic"],
                    "launches": d["launches"], "avg_launch_us": d["avg_launch_us"],
                    "algorithmic_bytes_per_launch": d["algorithmic_bytes_per_launch"]})
    else:
        # the local Newton solves have a data-dependent iteration count: no algorithmic operation
        # count per launch is fixed for them (their FP64 VALU rate is taken from counters)
        n, ms, units = fam[dom]
        out.update({"bound": "alu", "achieved": None, "peak": 78.6, "unit": "TFLOP/s", "frac": None,
                    "traffic": None, "launches": n, "avg_launch_us": 1e3 * ms / max(n, 1)})
    out["spectral_kernels"] = per
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
        print(json.dumps({"error": "this benchmark runs on one GPU only (this build has no multi-GPU "
                                   "path); run it with --gpus 1"}))
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
    opts = dict(newton_tol=NEWTON_TOL, cg_tol=CG_TOL, max_cg=3000, max_newton=150,
                use_graph=0 if args.no_graph else 1, autotune=0 if args.no_autotune else 1)
    # warmup once, in the mixed form
    h = lib.Homogenizer(rves, precision=lib.RVE_MIXED, **opts)
    for k in range(1, W + 1):
        h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        print(f"[mixed] warmup increment {k} done", file=sys.stderr, flush=True)
    state = h.save_state()
    mixed = timed(h, path, W + 1, K, "mixed")
    h.close()
    nvox = sum(r.n_vox for r in rves)
    config = {"workload": args.workload, "n_rve": len(rves), "voxels": nvox,
              "grids": sorted({tuple(r.n) for r in rves}), "increments_timed": [W + 1, W + K],
              "newton_tol": NEWTON_TOL, "cg_tol": CG_TOL, "precision": "mixed",
              "batching": {"rves_per_handle": len(rves), "host_workers": 8, "streams": len(rves),
                           "cg_chunks_as_hip_graphs": not args.no_graph, "autotuned_z_tiles": not args.no_autotune},
              "per_increment": mixed["per_increment"],
              "discarded_voxel_iterations": mixed["discarded_vi"],
              "fp64_fallbacks": sum(p["fp64_fallbacks"] for p in mixed["per_increment"]),
              "env": {k: os.environ[k] for k in ("RVE_PLANE", "RVE_TANGENT16", "RVE_PREDICT", "RVE_WORKERS",
                                                 "RVE_TZ", "GPU_MAX_HW_QUEUES") if k in os.environ}}
    if not args.no_fp64_compare:
        h = lib.Homogenizer(rves, precision=lib.RVE_FP64, **opts)
        h.load_state(state)
        ref = timed(h, path, W + 1, K, "fp64")
        h.close()
        import numpy as np
        Pm, Pf = np.array(mixed["P11"]), np.array(ref["P11"])
        rel = np.max(np.abs(Pm - Pf), axis=0) / np.max(np.abs(Pf), axis=0)   # per RVE, over increments
        config["fp64_form"] = {"value": ref["vi"] / ref["T"], "ms_per_step": 1e3 * ref["T"] / K,
                               "time_ratio_fp64_over_mixed": ref["T"] / mixed["T"],
                               "per_increment": ref["per_increment"],
                               "discarded_voxel_iterations": ref["discarded_vi"],
                               "P11_rel_diff_mixed_vs_fp64": float(rel.max()),
                               "P11_rel_diff_per_rve": [float("%.3g" % v) for v in rel],
                               "start": "the same saved state after the mixed warmup"}
    line = {
        "metric": METRIC,
        "value": mixed["vi"] / mixed["T"],
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * mixed["T"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32+f16",
        "data": "synthetic",
        "config": config,
    }
    if not args.no_roofline:
        fam, T = roofline_replay(lib, rves, path, state, W + 1, max(1, min(args.replay, K)), opts)
        line["roofline"] = roofline(fam, T, args.workload)
    del state
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, len(rves))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
