"""rve_project_noalloc: the projection of eq. 17 with the library's fixed scratch array, against
rve_project (GPU only).  Two calls in a row, the second on a smaller grid, so that the second
call finds the first call's tables and spectrum left in the shared array."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_01946_amd as m
    m.lib()
    return m


def _abi_project(L, fn, n, precision, A, mask, dc, out):
    nn = (ctypes.c_int32 * 3)(*n)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    dcp = None if dc is None else np.ascontiguousarray(dc, dtype=np.float64)
    rc = getattr(L, fn)(nn, precision, ctypes.c_void_p(A.data_ptr()), m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                        None if dcp is None else dcp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        ctypes.c_void_p(out.data_ptr()), None)
    assert rc == 0, L.rve_last_error()


@pytest.mark.parametrize("precision,bar", [(0, 1e-13), (1, 2e-6)])
def test_noalloc_projection_equals_rve_project_on_two_calls(lib, precision, bar):
    import torch
    L = lib.lib()
    mask = synth.UNIAXIAL_MASK
    dc = np.linspace(-1.0, 1.0, 9)
    for call, n in enumerate(((40, 48, 24), (16, 12, 10))):
        print(f"no-alloc projection call {call + 1}: grid {n}, precision {precision}", flush=True)
        V = n[0] * n[1] * n[2]
        A = torch.from_numpy(synth.random_field(700 + call, (9, V))).to("cuda:0")
        ref = torch.zeros_like(A)
        got = torch.full_like(A, float("nan"))
        _abi_project(L, "rve_project", n, precision, A, mask, dc, ref)
        _abi_project(L, "rve_project_noalloc", n, precision, A, mask, dc, got)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.isfinite(g).all()
        err = np.linalg.norm(g - r) / np.linalg.norm(r)
        print(f"  relative difference {err:.2e} (bar {bar:g})", flush=True)
        assert err <= bar
