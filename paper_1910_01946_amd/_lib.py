"""ctypes declarations of the C ABI in include/rve.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librve.so")

RVE_OK, RVE_EINVAL, RVE_ENOMEM, RVE_EDEVICE, RVE_ENOCONV, RVE_ESTATE = 0, -1, -2, -3, -4, -5
RVE_FP64, RVE_MIXED = 0, 1
STATUS_NAMES = {0: "RVE_OK", -1: "RVE_EINVAL", -2: "RVE_ENOMEM", -3: "RVE_EDEVICE", -4: "RVE_ENOCONV",
                -5: "RVE_ESTATE"}


class rve_material(C.Structure):
    _fields_ = [("C11", C.c_double), ("C12", C.c_double), ("C44", C.c_double), ("mu", C.c_double),
                ("burgers", C.c_double), ("y_c", C.c_double), ("K_sim", C.c_double),
                ("gamma0_dot", C.c_double), ("m_rate", C.c_double), ("q", C.c_double * 6),
                ("tau0", C.c_double), ("rho0", C.c_double), ("c_gnd", C.c_double),
                ("hardening", C.c_int32)]


class rve_desc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("voxel_size", C.c_double), ("n_grains", C.c_int32),
                ("grain_of_voxel", C.POINTER(C.c_int32)), ("grain_quat", C.POINTER(C.c_double)),
                ("material", rve_material), ("grain_elastic", C.POINTER(C.c_double))]


class rve_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("newton_tol", C.c_double), ("cg_tol", C.c_double),
                ("max_newton", C.c_int32), ("max_cg", C.c_int32), ("max_backtrack", C.c_int32),
                ("device", C.c_int32), ("stream", C.c_void_p), ("use_graph", C.c_int32),
                ("workers", C.c_int32), ("autotune", C.c_int32), ("max_cutbacks", C.c_int32),
                ("max_continuation", C.c_int32), ("frequencies", C.c_int32),
                ("projection", C.c_int32)]


class rve_step_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_iters", C.c_int32), ("cg_iters", C.c_int32),
                ("residual_evals", C.c_int32), ("line_search_cuts", C.c_int32),
                ("local_iters_max", C.c_int32), ("res_norm", C.c_double), ("dF_norm", C.c_double),
                ("voxel_iterations", C.c_double), ("fp64_fallback", C.c_int32),
                ("continuation_stages", C.c_int32), ("discarded_voxel_iterations", C.c_double),
                ("cutbacks", C.c_int32), ("pad", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """The loaded HIP library; raises LibraryMissing when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} not found: build it with __graft_entry__.build() "
                             "(or python paper_1910_01946_amd/build.py)")
    # torch brings its own HIP runtime; loading it first makes the library bind to that
    # same runtime instead of initialising a second one in the process
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp = C.c_void_p
    dp = P(C.c_double)
    L.rve_create.argtypes = [P(rve_desc), C.c_int32, P(rve_options), P(vp)]
    L.rve_create.restype = C.c_int32
    L.rve_step_increment.argtypes = [vp, dp, P(C.c_uint8), dp, C.c_double, P(rve_step_stats)]
    L.rve_step_increment.restype = C.c_int32
    L.rve_nye_gnd.argtypes = [vp, C.c_int32, dp, dp]
    L.rve_nye_gnd.restype = C.c_int32
    L.rve_macro_stress.argtypes = [vp, C.c_int32, dp, dp, dp]
    L.rve_macro_stress.restype = C.c_int32
    L.rve_get_field.argtypes = [vp, C.c_int32, C.c_int32, dp]
    L.rve_get_field.restype = C.c_int32
    L.rve_state_bytes.argtypes = [vp]
    L.rve_state_bytes.restype = C.c_int64
    L.rve_save_state.argtypes = [vp, vp]
    L.rve_save_state.restype = C.c_int32
    L.rve_load_state.argtypes = [vp, vp]
    L.rve_load_state.restype = C.c_int32
    L.rve_destroy.argtypes = [vp]
    L.rve_destroy.restype = None
    L.rve_last_error.argtypes = []
    L.rve_last_error.restype = C.c_char_p
    L.rve_constitutive_batch.argtypes = [P(rve_material), C.c_int32, dp, C.c_int64, vp, vp, vp, vp, vp,
                                         C.c_double, vp, vp, vp, vp, vp]
    L.rve_constitutive_batch.restype = C.c_int32
    L.rve_project.argtypes = [P(C.c_int32), C.c_int32, vp, P(C.c_uint8), dp, vp, vp]
    L.rve_project.restype = C.c_int32
    L.rve_project_noalloc.argtypes = [P(C.c_int32), C.c_int32, vp, P(C.c_uint8), dp, vp, vp]
    L.rve_project_noalloc.restype = C.c_int32
    L.rve_spectral_curl.argtypes = [P(C.c_int32), C.c_int32, C.c_double, vp, vp, vp, C.c_int32, dp,
                                    C.c_double, vp, vp]
    L.rve_spectral_curl.restype = C.c_int32
    L.rve_gnd_adjoint.argtypes = [P(C.c_int32), C.c_int32, C.c_double, vp, vp, C.c_int32, dp, C.c_double,
                                  vp, vp, vp, vp]
    L.rve_gnd_adjoint.restype = C.c_int32
    L.rve_stress_sensitivity.argtypes = [P(rve_material), C.c_int32, dp, C.c_int64, vp, vp, vp, vp, vp, C.c_double,
                                         vp, vp, vp]
    L.rve_stress_sensitivity.restype = C.c_int32
    L.rve_stress_sensitivity_vjp.argtypes = [P(rve_material), C.c_int32, dp, C.c_int64, vp, vp, vp, vp, vp,
                                             C.c_double, vp, vp, vp, vp]
    L.rve_stress_sensitivity_vjp.restype = C.c_int32
    L.rve_density_sensitivity.argtypes = [P(rve_material), C.c_int64, vp, vp, vp, vp, vp]
    L.rve_density_sensitivity.restype = C.c_int32
    L.rve_timing_start.argtypes = [vp, C.c_uint32]
    L.rve_timing_start.restype = C.c_int32
    L.rve_timing_read.argtypes = [vp, C.c_int32, P(C.c_int64), dp, dp]
    L.rve_timing_read.restype = C.c_int32
    L.rve_adjoint_solve.argtypes = [vp, C.c_int32, P(C.c_uint8), vp, vp, P(C.c_int32)]
    L.rve_adjoint_solve.restype = C.c_int32
    L.rve_adjoint_increment.argtypes = [vp, C.c_int32, P(C.c_uint8), dp, vp, vp, dp, P(C.c_int32)]
    L.rve_adjoint_increment.restype = C.c_int32
    _lib = L
    return L


# names the C ABI exports (checked by the CPU test suite)
EXPORTS = ["rve_create", "rve_step_increment", "rve_nye_gnd", "rve_macro_stress", "rve_get_field",
           "rve_state_bytes", "rve_save_state", "rve_load_state", "rve_destroy", "rve_last_error",
           "rve_constitutive_batch", "rve_project", "rve_project_noalloc", "rve_spectral_curl", "rve_timing_start",
           "rve_timing_read", "rve_adjoint_solve", "rve_adjoint_increment", "rve_gnd_adjoint",
           "rve_stress_sensitivity", "rve_stress_sensitivity_vjp", "rve_density_sensitivity"]

# kernel families of rve_timing_start / rve_timing_read
KERNEL_FAMILIES = {"slip_fast": 0, "slip_slow": 1, "stress_tangent": 2, "cg_prep": 3, "plane_fwd": 4, "mid": 5,
                   "plane_inv": 6, "cg_grad": 7, "plane_div": 8, "mid3": 9, "plane_w": 10}


class RVEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(rc):
    if rc != RVE_OK:
        raise RVEError(rc, lib().rve_last_error().decode())
    return rc
