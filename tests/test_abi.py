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
