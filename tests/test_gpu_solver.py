"""End-to-end parity of rve_step_increment against the oracle (GPU only)."""
import numpy as np
import pytest

import synth
from oracle import solver
from tests.gpu_util import from_abi, rel_norm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_01946_amd as m
    m.lib()
    return m


def _run_both(lib, rve, path, n_inc, precision=0, newton_tol=1e-11, cg_tol=1e-10):
    o = solver.RVESolver(rve, newton_tol=newton_tol, cg_tol=cg_tol)
    h = lib.Homogenizer([rve], precision=precision, newton_tol=newton_tol, cg_tol=cg_tol, max_cg=4000)
    out = []
    for k in range(1, n_inc + 1):
        print(f"increment {k} of {rve.n} precision={precision}", flush=True)
        so = o.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        assert so["converged"], so
        sg = h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)[0]
        print("  oracle", {k2: so[k2] for k2 in ("newton", "cg", "residuals")}, "gpu",
              {k2: sg[k2] for k2 in ("newton_iters", "cg_iters", "residual_evals", "local_iters_max")}, flush=True)
        Po, Fo, _ = o.macro()
        Pg, Fg, _ = h.macro()
        out.append((Po, Pg, Fo, Fg))
    return o, h, out


@pytest.mark.parametrize("plane", ["1", "0"])
def test_cu16_at_8cubed_fp64_matches_oracle(lib, plane, monkeypatch):
    monkeypatch.setenv("RVE_PLANE", plane)
    rves, path = synth.workload("cu16", n_override=8, n_inc_override=20)
    o, h, out = _run_both(lib, rves[0], path, 3)
    for Po, Pg, Fo, Fg in out:
        scale = np.abs(Po).max()
        assert np.max(np.abs(Pg - Po)) <= 1e-10 * scale, (Pg, Po)
        assert np.max(np.abs(Fg - Fo)) <= 1e-12
    V = rves[0].n_vox
    assert rel_norm(from_abi(h.field("F")), o.F) < 1e-11
    assert rel_norm(from_abi(h.field("P")), o.P) < 1e-10
    assert rel_norm(from_abi(h.field("Fp")), o.Fp) < 1e-12
    assert rel_norm(from_abi(h.field("rho_ssd"), tensor=False), o.rho_ssd) < 1e-10


def test_cu64_sgcp_at_8cubed_fp64_matches_oracle(lib):
    rves, path = synth.workload("cu64", n_override=8, n_inc_override=50)
    o, h, out = _run_both(lib, rves[0], path, 3)
    for Po, Pg, Fo, Fg in out:
        assert np.max(np.abs(Pg - Po)) <= 1e-10 * np.abs(Po).max()
    assert rel_norm(from_abi(h.field("nye")), o.alpha) < 1e-10
    assert rel_norm(from_abi(h.field("rho_gnd"), tensor=False), o.rho_gnd) < 1e-10
