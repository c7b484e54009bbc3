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
    ap.add_argument("--profiles-dir", default=None, help="where the summaries go (default: profiles/)")
    ap.add_argument("--bench-json", default=None, help="an unprofiled bench line to compare with (--summarize-trace)")
    ap.add_argument("--summarize-trace", default=None, metavar="DIR",
                    help="write profiles/kernels_* from the kernel trace under DIR (see TRACE_RUNS)")
    ap.add_argument("--summarize-counters", default=None, metavar="DIR",
                    help="write profiles/pmc_* from the counter runs under DIR (see COUNTER_RUNS)")
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
    """Ratio of measured HBM bytes (FETCH_SIZE and WRITE_SIZE, each scaled by the reading of a
    plain copy) to algorithmic bytes per launch, from the committed counter summary of this kernel
    and workload; None when the summary is missing or the kernel's sources changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_{family}_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^traffic_ratio\s*=\s*([0-9.eE+]+)", text, re.M)
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


def _load_roctx():
    """The profiler-control entry points (rocprofiler-sdk's tracer library; the older libroctx64,
    also bundled with torch, lacks them), loaded before HIP starts so that a profiler in the
    process registers them; None when absent."""
    import ctypes

    for name in ("/opt/rocm/lib/librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so.1"):
        try:
            L = ctypes.CDLL(name)
            L.roctxProfilerResume.argtypes = [ctypes.c_uint64]
            L.roctxProfilerPause.argtypes = [ctypes.c_uint64]
            return L
        except (OSError, AttributeError):
            continue
    return None


_ROCTX = None


class ProfilerRegion:
    """The serialised replay, marked for profilers: roctxProfilerResume(0) before it and
    roctxProfilerPause(0) after it (for rocprofv3 --selected-regions; no effect without a
    profiler), and one fill kernel (a torch.full) right before its first launch, after which a
    trace or counter run of the whole process is summarised."""

    def __enter__(self):
        import torch

        if _ROCTX is not None:
            _ROCTX.roctxProfilerResume(0)
        # marker for a trace of the whole process: one fill kernel right before the replay
        torch.full((1,), 7.0, device="cuda")
        torch.cuda.synchronize()
        return self

    def __exit__(self, *exc):
        if _ROCTX is not None:
            _ROCTX.roctxProfilerPause(0)
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
                    "traffic": None})
        ratio = stored_traffic(f, workload, "mixed")
        if ratio is not None:
            # measured / algorithmic bytes from the counter sample, applied to this replay's launches
            per[-1]["traffic"] = ratio * units / n
            per[-1]["traffic_ratio"] = ratio
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
    # the constitutive kernels against the FP64 vector peak (flops per launch from counters)
    cons = []
    for _, f in CONST_FAMILIES:
        n, ms, units = fam[f]
        if n == 0:
            continue
        # the continuation pass works through a data-dependent list with a fixed grid: no flops per
        # voxel apply to it
        fpv = stored_flops(f, workload) if f != "slip_slow" else None
        # units: voxels per launch (the listed voxels for the continuation pass)
        ach = fpv * units / (ms * 1e-3) / 1e12 if fpv else None
        cons.append({"family": f, "kernel": FAMILY_KERNELS[f][0], "bound": "alu", "launches": n,
                     "avg_launch_us": 1e3 * ms / n, "flops_per_voxel": fpv, "voxels_per_launch": units / n,
                     "achieved": ach,
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / FP64_PEAK_TFLOPS if ach else None, "share": round(share[f], 4)})
    out["constitutive_kernels"] = cons
    if dom not in SPECTRAL:
        d = next((c for c in cons if c["family"] == dom), None)
        if d and d["frac"] is not None:
            out.update({"achieved": d["achieved"], "frac": d["frac"]})
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


# Counter runs behind the committed summaries (from the repository root R on one MI355X; one host
# worker; only the dispatches after the replay marker are summarised):
COUNTER_RUNS = """cd /tmp && export TMPDIR=/tmp && export RVE_WORKERS=1
rocprofv3 --pmc FETCH_SIZE --output-format csv -d $R/gpurun_out/pmc_copy_f -o c -- python3 $R/bench.py --copy-calibration
rocprofv3 --pmc WRITE_SIZE --output-format csv -d $R/gpurun_out/pmc_copy_w -o c -- python3 $R/bench.py --copy-calibration
rocprofv3 --pmc FETCH_SIZE --kernel-include-regex "{regex}" --output-format csv -d $R/gpurun_out/pmc_f -o m -- python3 $R/bench.py {sample} --no-fp64-compare --no-cpu-baseline
rocprofv3 --pmc WRITE_SIZE --kernel-include-regex "{regex}" --output-format csv -d $R/gpurun_out/pmc_w -o m -- python3 $R/bench.py {sample} --no-fp64-compare --no-cpu-baseline > $R/gpurun_out/pmc_w_bench.json
rocprofv3 --pmc SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU_FLOPS_FP64 SQ_INSTS_VALU SQ_BUSY_CYCLES --kernel-include-regex "FillFunctor|k_slip_fast|k_slip_slow|k_stress_tangent" --output-format csv -d $R/gpurun_out/pmc_valu -o m -- python3 $R/bench.py {sample} --no-fp64-compare --no-cpu-baseline
python3 bench.py --summarize-counters gpurun_out --profiles-dir gpurun_out/summaries   (then copied to profiles/)"""
CONST_FAMILIES = (("k_slip_fast", "slip_fast"), ("k_slip_slow", "slip_slow"), ("k_stress_tangent<", "stress_tangent"))
FP64_PEAK_TFLOPS = 78.6
SPECTRAL_REGEX = "FillFunctor|k_cg_prep|k_plane_fwd|k_mid|k_plane_inv|k_cg_grad"
# Counter collection serialises every dispatch: the counter runs take a sample of the workload
# (its first four RVEs, the same warmup, one replayed increment), and the summaries keep the ratio of
# measured to algorithmic bytes, which the bench applies to its own replay's launches.
COUNTER_SAMPLE = "--rves 4 --warmup 5 --steps 1 --replay 1"
# template arguments that tell the spectral families apart in the demangled kernel names
# (PF_F64 = 1, PF_DIV = 3; MID_GREEN = 0, MID_GREEN3 = 2; PI_RESID = 1, PI_OUT_T = 3)
_NAME_FAMILY = [(r"k_cg_prep<float, 1, 0>", "cg_prep"), (r"k_plane_fwd<float, 3,", "plane_div"),
                (r"k_plane_fwd<float, 1,", "plane_fwd"), (r"k_mid<float, 2,", "mid3"), (r"k_mid<float, 0,", "mid"),
                (r"k_plane_inv<float, 3,", "plane_w"), (r"k_plane_inv<float, 1,", "plane_inv"),
                (r"k_cg_grad<float>", "cg_grad")]


def _counter_rows(directory, after_marker=True, with_grid=False):
    """(kernel name, counter, value) of the dispatches in the rocprofv3 CSV files under directory;
    with after_marker, only those after the last replay marker (the fill kernel that bench.py
    launches right before its serialised replay)."""
    import csv
    import glob

    rows = []
    for f in glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                did = int(r.get("Dispatch_Id") or r.get("Correlation_Id") or 0)
                rows.append((did, r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]),
                             int(float(r.get("Grid_Size") or 0))))
    rows.sort(key=lambda t: t[0])
    if after_marker:
        marks = [r[0] for r in rows if "FillFunctor" in r[1]]
        if not marks:
            raise SystemExit(f"no replay marker among the dispatches under {directory}")
        rows = [r for r in rows if r[0] > max(marks)]
    return [r[1:] if with_grid else r[1:4] for r in rows]


def summarize_counters(out_dir, workload="sweep32", profiles=None):
    """Write profiles/pmc_<family>_<workload>_mixed.txt for every spectral family found in the
    counter runs of COUNTER_RUNS: FETCH_SIZE and WRITE_SIZE per live dispatch (a dispatch that a
    finished CG solve turned into a no-op reads and writes a few KiB; live ones at least
    hundreds), each scaled by the same counter's reading of a 2^30-byte copy, against the
    algorithmic bytes per launch that the bench line of the WRITE_SIZE run reports."""
    import numpy as np

    def copy_scale(d, counter):
        vals = [v for k, c, v in _counter_rows(d, after_marker=False) if c == counter and "copy" in k.lower()]
        if not vals:
            raise SystemExit(f"no copy dispatches with {counter} under {d}")
        return (1 << 30) / (1024.0 * float(np.median(vals))), float(np.median(vals))

    if profiles:
        os.makedirs(profiles, exist_ok=True)
    s_f, kib_f = copy_scale(os.path.join(out_dir, "pmc_copy_f"), "FETCH_SIZE")
    s_w, kib_w = copy_scale(os.path.join(out_dir, "pmc_copy_w"), "WRITE_SIZE")
    line = json.loads(open(os.path.join(out_dir, "pmc_w_bench.json")).read().strip().splitlines()[-1])
    alg = {p["family"]: p for p in line["roofline"]["spectral_kernels"]}
    per = {}
    for counter, d in (("FETCH_SIZE", "pmc_f"), ("WRITE_SIZE", "pmc_w")):
        for name, c, v in _counter_rows(os.path.join(out_dir, d)):
            if c != counter:
                continue
            fam = next((f for pat, f in _NAME_FAMILY if pat in name), None)
            if fam:
                per.setdefault(fam, {}).setdefault(counter, []).append(v)
    written = []
    for fam, cs in sorted(per.items()):
        if fam not in alg or "FETCH_SIZE" not in cs or "WRITE_SIZE" not in cs:
            continue
        live = {c: [v for v in vals if v > 64.0] for c, vals in cs.items()}
        f_mb = 1024.0 * s_f * float(np.mean(live["FETCH_SIZE"])) / 1e6
        w_mb = 1024.0 * s_w * float(np.mean(live["WRITE_SIZE"])) / 1e6
        a = alg[fam]
        traffic = (f_mb + w_mb) * 1e6
        text = f"""# HBM traffic of {a['instantiation']} on the {workload} workload, mixed form
# (counter sample: {COUNTER_SAMPLE}, serialised, one RVE at a time; per-launch figures are averages
# over the live launches of the replayed increment)

commands (repository root R, one MI355X), one counter per run:
{COUNTER_RUNS.format(regex=SPECTRAL_REGEX, sample=COUNTER_SAMPLE)}

calibration: a device copy of 2^30 bytes, 5 dispatches
  FETCH_SIZE {kib_f:.1f} KiB per dispatch for 1048576 KiB read     -> scale {s_f:.5f}
  WRITE_SIZE {kib_w:.1f} KiB per dispatch for 1048576 KiB written  -> scale {s_w:.5f}

{a['instantiation']}: FETCH_SIZE {len(cs['FETCH_SIZE'])} dispatches ({len(live['FETCH_SIZE'])} live), WRITE_SIZE {len(cs['WRITE_SIZE'])} ({len(live['WRITE_SIZE'])} live); the bench's events counted {a['launches']} live launches
  FETCH_SIZE live mean -> {f_mb:.3f} MB read per launch
  WRITE_SIZE live mean -> {w_mb:.3f} MB written per launch
  algorithmic bytes per launch (bench line of the WRITE_SIZE run): {a['algorithmic_bytes_per_launch'] / 1e6:.3f} MB; measured / algorithmic = {traffic / a['algorithmic_bytes_per_launch']:.2f}

traffic_bytes_per_launch = {traffic:.0f}
traffic_ratio = {traffic / a['algorithmic_bytes_per_launch']:.4f}
source_digest = {source_digest(FAMILY_KERNELS[fam][1])}
"""
        path = os.path.join(profiles or os.path.join(ROOT, "profiles"), f"pmc_{fam}_{workload}_mixed.txt")
        with open(path, "w") as fh:
            fh.write(text)
        written.append((fam, traffic / a["algorithmic_bytes_per_launch"]))
    # FP64 vector work of the constitutive kernels: 64 lanes x (2 FMA + ADD + MUL + TRANS) per
    # wave instruction (no MFMA on this path), per dispatch
    vrows = _counter_rows(os.path.join(out_dir, "pmc_valu"), with_grid=True)
    if vrows:
        by, grid = {}, {}
        for name, c, v, gs in vrows:
            fam = next((f for pat, f in CONST_FAMILIES if pat in name), None)
            if fam:
                by.setdefault(fam, {}).setdefault(c, []).append(v)
                if c == "SQ_INSTS_VALU_FMA_F64":
                    grid.setdefault(fam, []).append(gs)
        lines = [f"# FP64 vector work of the constitutive kernels on the {workload} workload, mixed form",
                 "# (serialised replay of two increments from the saved state, every dispatch)", "",
                 "commands (repository root R, one MI355X):", COUNTER_RUNS.format(regex=SPECTRAL_REGEX, sample=COUNTER_SAMPLE), "",
                 "flops per dispatch = 64 x (2 SQ_INSTS_VALU_FMA_F64 + SQ_INSTS_VALU_ADD_F64 + SQ_INSTS_VALU_MUL_F64"
                 " + SQ_INSTS_VALU_TRANS_F64) (all lanes active); SQ_INSTS_VALU_FLOPS_FP64 is the hardware's own count;",
                 "flops per voxel = flops per dispatch / threads per dispatch (one voxel per thread; k_slip_slow",
                 "runs a fixed grid over the list of voxels the first pass left, so its figure is per grid thread)", ""]
        for fam, cs in sorted(by.items()):
            n = len(cs.get("SQ_INSTS_VALU_FMA_F64", []))
            if not n:
                continue
            m = {c: float(np.mean(v)) for c, v in cs.items()}
            fl = 64.0 * (2 * m.get("SQ_INSTS_VALU_FMA_F64", 0) + m.get("SQ_INSTS_VALU_ADD_F64", 0) +
                         m.get("SQ_INSTS_VALU_MUL_F64", 0) + m.get("SQ_INSTS_VALU_TRANS_F64", 0))
            fp64_share = (m.get("SQ_INSTS_VALU_FMA_F64", 0) + m.get("SQ_INSTS_VALU_ADD_F64", 0) +
                          m.get("SQ_INSTS_VALU_MUL_F64", 0) + m.get("SQ_INSTS_VALU_TRANS_F64", 0)) / max(m.get("SQ_INSTS_VALU", 1), 1)
            fpv = float(np.sum([64.0 * (2 * a + b + c + d) for a, b, c, d in zip(
                cs.get("SQ_INSTS_VALU_FMA_F64", []), cs.get("SQ_INSTS_VALU_ADD_F64", [0] * n),
                cs.get("SQ_INSTS_VALU_MUL_F64", [0] * n), cs.get("SQ_INSTS_VALU_TRANS_F64", [0] * n))])
                        / max(float(np.sum(grid.get(fam, [1]))), 1.0))
            lines += [f"{fam}: {n} dispatches",
                      f"  mean per dispatch: FMA_F64 {m.get('SQ_INSTS_VALU_FMA_F64', 0):.4g}, ADD_F64 {m.get('SQ_INSTS_VALU_ADD_F64', 0):.4g}, "
                      f"MUL_F64 {m.get('SQ_INSTS_VALU_MUL_F64', 0):.4g}, TRANS_F64 {m.get('SQ_INSTS_VALU_TRANS_F64', 0):.4g}, "
                      f"VALU {m.get('SQ_INSTS_VALU', 0):.4g} wave instructions; FLOPS_FP64 counter {m.get('SQ_INSTS_VALU_FLOPS_FP64', 0):.4g}",
                      f"  FP64 share of the VALU instructions {fp64_share:.3f}",
                      f"flops_per_launch_{fam} = {fl:.6g}",
                      f"flops_per_voxel_{fam} = {fpv:.6g}", ""]
        lines.append(f"source_digest = {source_digest(_CONST_SRC)}")
        with open(os.path.join(profiles or os.path.join(ROOT, "profiles"), f"pmc_valu_constitutive_{workload}_mixed.txt"),
                  "w") as fh:
            fh.write("\n".join(lines) + "\n")
        written.append(("constitutive", None))
    print(json.dumps({"written": written}))


def stored_flops(family: str, workload: str):
    """FP64 flops per voxel of a constitutive kernel's launch from the committed VALU counter
    summary; None when missing or the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"pmc_valu_constitutive_{workload}_mixed.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(rf"^flops_per_voxel_{family}\s*=\s*([0-9.eE+]+)", text, re.M)
    d = re.search(r"^source_digest\s*=\s*([0-9a-f]+)", text, re.M)
    if not m or not d or d.group(1) != source_digest(_CONST_SRC):
        return None
    return float(m.group(1))


TRACE_RUNS = """cd /tmp && export TMPDIR=/tmp && export RVE_WORKERS=1
rocprofv3 --kernel-trace --stats --output-format csv -d $R/gpurun_out/trace_replay -o replay -- python3 $R/bench.py --steps 1 --warmup 5 --replay 2 --no-fp64-compare --no-cpu-baseline > $R/gpurun_out/trace_replay.json
python3 bench.py --summarize-trace gpurun_out --profiles-dir gpurun_out/summaries --bench-json gpurun_out/bench.json   (bench.json: the unprofiled default run; then copied to profiles/)"""
def summarize_trace(out_dir, workload="sweep32", profiles=None, bench_json=None):
    """profiles/kernels_<workload>_mixed_replay.txt from the kernel trace of TRACE_RUNS: per
    family, the dispatches after the replay marker, their total time, and the mean over the live
    ones against the event-timed figures that the traced process printed.  A CG launch issued
    after its solve converged reads the stop flag and returns within about 2 us; the event timer
    knows how many launches were live, so the shortest (dispatches - live) dispatches of a family
    are taken as its no-ops."""
    import csv
    import glob

    import numpy as np

    if profiles:
        os.makedirs(profiles, exist_ok=True)
    rows = []
    for f in glob.glob(os.path.join(out_dir, "trace_replay", "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
    rows.sort()
    # the replay follows the marker kernel that bench.py launches right before it
    marks = [i for i, (_, _, n) in enumerate(rows) if "FillFunctor" in n]
    if not marks:
        raise SystemExit("no replay marker in the trace")
    rows = rows[marks[-1] + 1:]
    line = json.loads(open(os.path.join(out_dir, "trace_replay.json")).read().strip().splitlines()[-1])
    roof = line["roofline"]
    ev = {p["family"]: p for p in roof["spectral_kernels"] + roof.get("constitutive_kernels", [])}
    # the same replay timed by an unprofiled bench run (the tracer slows the traced process's
    # own event timing by several us per launch)
    ub = {}
    if bench_json:
        r2 = json.loads(open(bench_json).read().strip().splitlines()[-1])["roofline"]
        ub = {p["family"]: p for p in r2["spectral_kernels"] + r2.get("constitutive_kernels", [])}
    names = _NAME_FAMILY + [(pat, f) for pat, f in CONST_FAMILIES]
    dur = {}
    for a, b, n in rows:
        fam = next((f for pat, f in names if pat in n), None)
        if fam:
            dur.setdefault(fam, []).append((b - a) / 1e3)
    inc = roof["replay_increments"]
    out = [f"# Kernel durations of the serialised replay ({workload}, mixed form, increments {inc[0]}-{inc[1]},",
           "# one RVE at a time, every RVE of the workload)", "",
           "commands (repository root R, one MI355X):", TRACE_RUNS, "",
           "per family: dispatches after the replay marker; live = those the event timer counted (the",
           "shortest dispatches - live are the no-op launches past a converged CG solve); trace mean over",
           "the live dispatches; the same launches timed with HIP events by the traced process and by an",
           "unprofiled bench run (bench mean); the algorithmic bytes per launch and the HBM fraction from",
           "the trace's duration", "",
           "family          dispatches   live  trace total ms  trace mean us  event mean us  bench mean us  "
           "noop max us  live min us  MB/launch  trace frac"]
    for fam in [f for f in SPECTRAL + tuple(f for _, f in CONST_FAMILIES) if f in dur]:
        d = np.sort(np.array(dur[fam]))
        e = ev.get(fam)
        n_live = min(len(d), e["launches"]) if e else len(d)
        noop, live = d[: len(d) - n_live], d[len(d) - n_live:]
        mb = e.get("algorithmic_bytes_per_launch", 0) / 1e6 if e else 0
        frac = mb * 1e6 / (live.mean() * 1e-6) / (HBM_PEAK_GBS * 1e9) if mb else float("nan")
        b = ub.get(fam)
        out.append(f"{fam:15s} {len(d):10d} {n_live:6d} {d.sum() / 1e3:15.2f} {live.mean():14.2f} "
                   f"{(e['avg_launch_us'] if e else float('nan')):14.2f} {(b['avg_launch_us'] if b else float('nan')):14.2f} "
                   f"{(noop.max() if len(noop) else float('nan')):12.2f} "
                   f"{live.min():12.2f} {mb:10.3f} {frac:11.3f}")
    text = "\n".join(out) + "\n"
    path = os.path.join(profiles or os.path.join(ROOT, "profiles"), f"kernels_{workload}_mixed_replay.txt")
    with open(path, "w") as fh:
        fh.write(text)
    print(text)


def main():
    global _ROCTX
    args = parse()
    _ROCTX = _load_roctx()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.workload, args.profiles_dir)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.workload, args.profiles_dir, args.bench_json)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the library has no multi-GPU "
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
              "batching": {"rves_per_handle": len(rves), "host_workers": int(os.environ.get("RVE_WORKERS", 8)), "streams": len(rves),
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
        Rn = max(1, min(args.replay, K))
        fam, T = roofline_replay(lib, rves, path, state, W + 1, Rn, opts)
        line["roofline"] = roofline(fam, T, args.workload)
        line["roofline"]["replay_increments"] = [W + 1, W + Rn]
    del state
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, len(rves))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
