"""The C-ABI library loads and exports every declared entry point (CPU, no compute)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rve.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rve_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for n in ("rve_create", "rve_step_increment", "rve_nye_gnd", "rve_macro_stress"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1910_01946_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("librve.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name
    assert sorted(_lib.EXPORTS) == declared_functions()


def test_binding_fails_loudly_without_library(monkeypatch):
    from paper_1910_01946_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/librve.so")
    with pytest.raises(_lib.LibraryMissing):
        _lib.lib()


def test_gnd_adjoint_rejects_bad_arguments_before_any_device_call():
    """The argument checks of rve_gnd_adjoint run on the host: no GPU is needed to see them."""
    from paper_1910_01946_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    L = _lib.lib()
    n = (ctypes.c_int32 * 3)(4, 4, 4)
    q = (ctypes.c_double * 4)(1.0, 0.0, 0.0, 0.0)
    fake = ctypes.c_void_p(16)   # never dereferenced: every call below fails its host checks
    cases = [
        (None, 1, 1.0, 0.25e-9, fake),    # null nye
        (fake, 0, 1.0, 0.25e-9, fake),    # no grains
        (fake, 1, 0.0, 0.25e-9, fake),    # h = 0
        (fake, 1, 1.0, -1.0, fake),       # negative Burgers vector
        (fake, 1, 1.0, 0.25e-9, None),    # null Fp_bar
    ]
    for nye, ng, h, b, out in cases:
        rc = L.rve_gnd_adjoint(n, 0, h, nye, fake, ng, q, b, fake, None, out, None)
        assert rc == -1
        assert L.rve_last_error()


def test_sensitivity_entry_points_reject_bad_arguments_before_any_device_call():
    """rve_stress_sensitivity and rve_density_sensitivity check their arguments and the
    material on the host: no GPU is needed to see the errors."""
    from paper_1910_01946_amd import _lib, make_material
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    import synth
    L = _lib.lib()
    good = make_material(synth.material("Cu"))
    bad = make_material(synth.material("Cu"))
    bad.burgers = -1.0
    q = (ctypes.c_double * 4)(1.0, 0.0, 0.0, 0.0)
    fake = ctypes.c_void_p(16)   # never dereferenced: every call below fails its host checks
    m = ctypes.byref(good)
    assert L.rve_stress_sensitivity(m, 1, q, 8, fake, fake, fake, fake, fake, 0.5, fake, None, None) == -1
    assert L.rve_stress_sensitivity(m, 1, q, 8, fake, fake, fake, fake, fake, 0.0, fake, fake, None) == -1
    assert L.rve_stress_sensitivity(m, 0, q, 8, fake, fake, fake, fake, fake, 0.5, fake, fake, None) == -1
    assert L.rve_density_sensitivity(m, 8, fake, fake, None, fake, None) == -1
    assert L.rve_density_sensitivity(m, 0, fake, fake, fake, fake, None) == -1
    assert L.rve_density_sensitivity(ctypes.byref(bad), 8, fake, fake, fake, fake, None) == -1
    assert L.rve_last_error()


def test_noalloc_projection_rejects_grids_beyond_its_scratch_array_on_the_host():
    """rve_project_noalloc checks the grid against its fixed 64 MiB scratch array before any
    device work: 128^3 in FP64 (a 153 MB spectrum) is refused with RVE_EINVAL, as are null
    pointers and bad grid sizes; no GPU is needed to see the errors."""
    from paper_1910_01946_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    L = _lib.lib()
    fake = ctypes.c_void_p(16)   # never dereferenced: every call below fails its host checks
    mask = (ctypes.c_uint8 * 9)(1, 1, 1, 1, 0, 1, 1, 1, 0)
    big = (ctypes.c_int32 * 3)(128, 128, 128)
    assert L.rve_project_noalloc(big, 0, fake, mask, None, fake, None) == -1
    assert b"too large" in L.rve_last_error()
    assert L.rve_project_noalloc(big, 1, fake, mask, None, fake, None) == -1   # 77 MB in FP32
    odd = (ctypes.c_int32 * 3)(14, 8, 8)  # prime factor 7
    assert L.rve_project_noalloc(odd, 0, fake, mask, None, fake, None) == -1
    ok = (ctypes.c_int32 * 3)(8, 8, 8)
    assert L.rve_project_noalloc(ok, 0, None, mask, None, fake, None) == -1
    assert L.rve_project_noalloc(ok, 2, fake, mask, None, fake, None) == -1
