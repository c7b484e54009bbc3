"""MI355X (gfx950) FFT strain-gradient crystal-plasticity homogenization.

Python binding of the C library (include/rve.h): argument marshalling only, every step
of the homogenization runs in the library's HIP kernels.  PyTorch supplies device memory
and streams for the kernel-level entry points.  There is no CPU fallback: without the
built library every call raises LibraryMissing.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (RVE_FP64, RVE_MIXED, LibraryMissing, RVEError, check, lib, rve_desc, rve_material,
                   rve_options, rve_step_stats)

__all__ = ["RVE_FP64", "RVE_MIXED", "Homogenizer", "make_material", "constitutive_batch", "project",
           "project_noalloc",
           "spectral_curl", "gnd_adjoint", "stress_sensitivity", "stress_sensitivity_vjp",
           "density_sensitivity",
           "LibraryMissing", "RVEError", "lib"]

FIELDS = {"F": (0, 9), "P": (1, 9), "Fp": (2, 9), "rho_ssd": (3, 12), "rho_gnd": (4, 12),
          "nye": (5, 9), "dg": (6, 12)}


def make_material(m) -> rve_material:
    """rve_material from any object with the synth.Material attributes."""
    out = rve_material()
    for k in ("C11", "C12", "C44", "mu", "burgers", "y_c", "K_sim", "gamma0_dot", "m_rate", "tau0",
              "rho0", "c_gnd"):
        setattr(out, k, float(getattr(m, k)))
    for i, v in enumerate(m.q):
        out.q[i] = float(v)
    out.hardening = int(m.hardening)
    return out


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Homogenizer:
    """A set of RVEs advanced together through rve_step_increment."""

    def __init__(self, rves, precision=RVE_FP64, newton_tol=1e-10, cg_tol=1e-8, max_newton=40,
                 max_cg=2000, max_backtrack=12, device=0, stream=None, use_graph=0, workers=0, autotune=0,
                 max_cutbacks=0, max_continuation=0, frequencies=0, projection=0):
        L = lib()
        n = len(rves)
        self._keep = []
        descs = (rve_desc * n)()
        for i, r in enumerate(rves):
            gid = np.ascontiguousarray(r.grain_of_voxel.reshape(-1), dtype=np.int32)
            q = np.ascontiguousarray(r.quats, dtype=np.float64)
            self._keep += [gid, q]
            d = descs[i]
            d.n[0], d.n[1], d.n[2] = (int(v) for v in r.n)
            d.voxel_size = float(r.voxel_size)
            d.n_grains = int(q.shape[0])
            d.grain_of_voxel = gid.ctypes.data_as(C.POINTER(C.c_int32))
            d.grain_quat = _dp(q)
            d.material = make_material(r.material)
            ge = getattr(r, "grain_elastic", None)
            if ge is not None:
                ge = np.ascontiguousarray(ge, dtype=np.float64).reshape(-1)
                self._keep.append(ge)
                d.grain_elastic = _dp(ge)
        opt = rve_options(precision=precision, newton_tol=newton_tol, cg_tol=cg_tol, max_newton=max_newton,
                          max_cg=max_cg, max_backtrack=max_backtrack, device=device,
                          stream=C.c_void_p(stream) if stream else None, use_graph=int(use_graph),
                          workers=int(workers), autotune=int(autotune), max_cutbacks=int(max_cutbacks),
                          max_continuation=int(max_continuation), frequencies=int(frequencies),
                          projection=int(projection))
        h = C.c_void_p()
        check(L.rve_create(descs, n, C.byref(opt), C.byref(h)))
        self.h = h
        self.rves = rves
        self.n_rve = n

    def close(self):
        if getattr(self, "h", None):
            lib().rve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, F_bar, mask, P_bar, dt):
        """One increment for every RVE; F_bar, P_bar: (9,) or (n_rve, 9).  Returns stats dicts."""
        F = np.ascontiguousarray(np.broadcast_to(np.asarray(F_bar, float).reshape(-1, 9), (self.n_rve, 9)))
        P = np.ascontiguousarray(np.broadcast_to(np.asarray(P_bar, float).reshape(-1, 9), (self.n_rve, 9)))
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(9))
        st = (rve_step_stats * self.n_rve)()
        rc = lib().rve_step_increment(self.h, _dp(F), m.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(P),
                                      float(dt), st)
        stats = [s.as_dict() for s in st]
        if rc != 0:
            err = RVEError(rc, lib().rve_last_error().decode())
            err.stats = stats
            raise err
        return stats

    def macro(self, i=0):
        P = np.zeros(9)
        F = np.zeros(9)
        s = np.zeros(9)
        check(lib().rve_macro_stress(self.h, i, _dp(P), _dp(F), _dp(s)))
        return P, F, s

    def field(self, name, i=0):
        which, nc = FIELDS[name]
        out = np.zeros((nc, self.rves[i].n_vox))
        check(lib().rve_get_field(self.h, i, which, _dp(out)))
        return out

    def nye_gnd(self, i=0):
        """rve_nye_gnd: the committed Nye tensor (9 x nvox, 1/m) and GND densities (12 x nvox,
        1/m^2) of RVE i, component-major."""
        n = self.rves[i].n_vox
        nye = np.zeros((9, n))
        rho = np.zeros((12, n))
        check(lib().rve_nye_gnd(self.h, i, _dp(nye), _dp(rho)))
        return nye, rho

    def timing_start(self, families=()):
        """Time the launches of the named kernel families (see _lib.KERNEL_FAMILIES) with
        HIP events from now on; an empty list stops timing.  Clears the accumulators."""
        mask = 0
        for f in families:
            mask |= 1 << _lib.KERNEL_FAMILIES[f]
        check(lib().rve_timing_start(self.h, mask))

    def timing_read(self, family):
        """(launches, total ms, units) of a family since timing_start; units are
        algorithmic bytes for the spectral families, voxels for the constitutive ones."""
        n = C.c_int64(0)
        t = C.c_double(0.0)
        u = C.c_double(0.0)
        check(lib().rve_timing_read(self.h, _lib.KERNEL_FAMILIES[family], C.byref(n), C.byref(t), C.byref(u)))
        return n.value, t.value, u.value

    def adjoint_solve(self, g, mask, lam, i=0):
        """Solve G(K^T : lam) = G(g) at the last increment of RVE i (rve_adjoint_solve).
        g, lam: device float64 tensors of 9 x nvox; returns the CG iteration count."""
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(9))
        n = C.c_int32(0)
        check(lib().rve_adjoint_solve(self.h, i, m.ctypes.data_as(C.POINTER(C.c_uint8)), _ptr(g), _ptr(lam),
                                      C.byref(n)))
        return n.value

    def adjoint_increment(self, mask, dLdP, Fp_bar, rho_bar, theta_bar, i=0):
        """Reverse pass of the last committed increment of RVE i (rve_adjoint_increment).
        dLdP: 9 host values; Fp_bar (9 x nvox), rho_bar (12 x nvox): device float64 tensors,
        updated in place; theta_bar: host float64 array of 4, accumulated.  Returns the CG
        iteration count of the multiplier solve."""
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(9))
        w = np.ascontiguousarray(np.asarray(dLdP, dtype=np.float64).reshape(9))
        assert theta_bar.dtype == np.float64 and theta_bar.flags.c_contiguous and theta_bar.size == 4
        n = C.c_int32(0)
        check(lib().rve_adjoint_increment(self.h, i, m.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(w), _ptr(Fp_bar),
                                          _ptr(rho_bar), _dp(theta_bar), C.byref(n)))
        return n.value

    def save_state(self):
        nb = lib().rve_state_bytes(self.h)
        buf = np.zeros(nb, dtype=np.uint8)
        check(lib().rve_save_state(self.h, buf.ctypes.data_as(C.c_void_p)))
        return buf

    def load_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        check(lib().rve_load_state(self.h, buf.ctypes.data_as(C.c_void_p)))


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    return C.c_void_p(stream) if stream else None


def constitutive_batch(mat, quats, gid, F, Fp_n, rho_ssd_n, rho_gnd_n, dt, dg, P, K=None, iters=None,
                       stream=None):
    """Kernel-level constitutive update on torch device tensors (component-major fields)."""
    q = np.ascontiguousarray(quats, dtype=np.float64)
    m = make_material(mat)
    check(lib().rve_constitutive_batch(C.byref(m), int(q.shape[0]), _dp(q), int(gid.numel()), _ptr(gid),
                                       _ptr(F), _ptr(Fp_n), _ptr(rho_ssd_n), _ptr(rho_gnd_n), float(dt),
                                       _ptr(dg), _ptr(P), _ptr(K), _ptr(iters), _stream(stream)))


def stress_sensitivity(mat, quats, gid, F, Fp_n, rho_ssd_n, rho_gnd_n, dt, dg, dPdtc, stream=None):
    """dPdtc (108 x nvox, row 9c + r) = dP_r / dtau_c,c at the slip increments dg (torch device
    tensors, component-major), for the adjoint form."""
    q = np.ascontiguousarray(quats, dtype=np.float64)
    m = make_material(mat)
    check(lib().rve_stress_sensitivity(C.byref(m), int(q.shape[0]), _dp(q), int(gid.numel()), _ptr(gid),
                                       _ptr(F), _ptr(Fp_n), _ptr(rho_ssd_n), _ptr(rho_gnd_n), float(dt),
                                       _ptr(dg), _ptr(dPdtc), _stream(stream)))


def stress_sensitivity_vjp(mat, quats, gid, F, Fp_n, rho_ssd_n, rho_gnd_n, dt, dg, w, tau_c_bar, stream=None):
    """tau_c_bar (12 x nvox) = sum_r w_r dP_r / dtau_c for an adjoint field w (9 x nvox), without
    forming the full sensitivity (torch device tensors, component-major)."""
    q = np.ascontiguousarray(quats, dtype=np.float64)
    m = make_material(mat)
    check(lib().rve_stress_sensitivity_vjp(C.byref(m), int(q.shape[0]), _dp(q), int(gid.numel()), _ptr(gid),
                                           _ptr(F), _ptr(Fp_n), _ptr(rho_ssd_n), _ptr(rho_gnd_n), float(dt),
                                           _ptr(dg), _ptr(w), _ptr(tau_c_bar), _stream(stream)))


def density_sensitivity(mat, rho_ssd_n, rho_gnd_n, dg, out, stream=None):
    """out (24 x nvox): d rho_SSD / dK (rows 0-11) and d rho_SSD / dy_c (rows 12-23) of the
    density update at fixed slip increments dg (torch device tensors, component-major)."""
    m = make_material(mat)
    check(lib().rve_density_sensitivity(C.byref(m), int(dg.shape[1]), _ptr(rho_ssd_n), _ptr(rho_gnd_n),
                                        _ptr(dg), _ptr(out), _stream(stream)))


def project(n, A, mask, out, dc_target=None, precision=RVE_FP64, stream=None):
    nn = (C.c_int32 * 3)(*[int(v) for v in n])
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(9))
    dc = None if dc_target is None else np.ascontiguousarray(np.asarray(dc_target, float).reshape(9))
    check(lib().rve_project(nn, precision, _ptr(A), m.ctypes.data_as(C.POINTER(C.c_uint8)),
                            _dp(dc) if dc is not None else None, _ptr(out), _stream(stream)))


def project_noalloc(n, A, mask, out, dc_target=None, precision=RVE_FP64, stream=None):
    """rve_project_noalloc: the projection with the library's fixed scratch array (no device
    allocation; asynchronous on stream)."""
    nn = (C.c_int32 * 3)(*[int(v) for v in n])
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(9))
    dc = None if dc_target is None else np.ascontiguousarray(np.asarray(dc_target, float).reshape(9))
    check(lib().rve_project_noalloc(nn, precision, _ptr(A), m.ctypes.data_as(C.POINTER(C.c_uint8)),
                                    _dp(dc) if dc is not None else None, _ptr(out), _stream(stream)))


def spectral_curl(n, h, Fp, nye, gid=None, quats=None, burgers=0.0, rho_gnd=None, precision=RVE_FP64,
                  stream=None):
    nn = (C.c_int32 * 3)(*[int(v) for v in n])
    q = None if quats is None else np.ascontiguousarray(quats, dtype=np.float64)
    check(lib().rve_spectral_curl(nn, precision, float(h), _ptr(Fp), _ptr(nye), _ptr(gid),
                                  0 if q is None else int(q.shape[0]), _dp(q) if q is not None else None,
                                  float(burgers), _ptr(rho_gnd), _stream(stream)))


def gnd_adjoint(n, h, nye, gid, quats, burgers, rho_bar, Fp_bar, nye_bar=None, precision=RVE_FP64,
                stream=None):
    """Fp_bar (and nye_bar when given) = transpose of d rho_GND / d Fp at the Nye tensor nye,
    applied to rho_bar; device tensors in the component-major layout of spectral_curl."""
    nn = (C.c_int32 * 3)(*[int(v) for v in n])
    q = np.ascontiguousarray(quats, dtype=np.float64)
    check(lib().rve_gnd_adjoint(nn, precision, float(h), _ptr(nye), _ptr(gid), int(q.shape[0]), _dp(q),
                                float(burgers), _ptr(rho_bar), _ptr(nye_bar), _ptr(Fp_bar), _stream(stream)))
