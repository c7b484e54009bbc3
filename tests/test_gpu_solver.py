"""End-to-end parity of rve_step_increment against the oracle (GPU only)."""
import numpy as np
import pytest

import synth
from oracle import constitutive, nye, solver
from tests.gpu_util import cuda, from_abi, rel_norm, to_abi

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
        # the FP64 bar of the parity contract (1e-10 relative on <P>); both solvers stop at
        # |dF| <= 1e-11 and agree to about 2e-13 (the oracle alone moves by 1e-13 when its
        # tolerances or its FFT axis order change)
        print("  <P> difference", np.max(np.abs(Pg - Po)) / scale, flush=True)
        assert np.max(np.abs(Pg - Po)) <= 1e-10 * scale, (Pg, Po)
        assert np.max(np.abs(Fg - Fo)) <= 1e-12
    V = rves[0].n_vox
    fields = {"F": rel_norm(from_abi(h.field("F")), o.F), "P": rel_norm(from_abi(h.field("P")), o.P),
              "Fp": rel_norm(from_abi(h.field("Fp")), o.Fp),
              "rho_ssd": rel_norm(from_abi(h.field("rho_ssd"), tensor=False), o.rho_ssd)}
    print("  field differences", fields, flush=True)
    assert fields["F"] < 1e-11
    assert fields["P"] < 1e-10
    assert fields["Fp"] < 1e-11
    assert fields["rho_ssd"] < 1e-10


def _check_gnd_fields(h, o, rve):
    """Nye tensor and GND densities: the kernels at 1e-12 on the GPU's own committed Fp; the
    whole increment at 1e-10 normwise, and below 10 x the measured Fp difference relative to
    |Fp - I| (the curl differentiates Fp - I, and the difference of two converged solutions
    is rougher than the field)."""
    Fp = from_abi(h.field("Fp"))
    d_fp = rel_norm(Fp, o.Fp)
    assert d_fp < 1e-11
    alpha, _, rho = nye.gnd_from_fp(Fp.reshape(rve.grain_of_voxel.shape + (3, 3)), rve.voxel_size,
                                    rve.grain_of_voxel, rve.quats, rve.material.burgers)
    assert rel_norm(from_abi(h.field("nye")), alpha.reshape(-1, 3, 3)) < 1e-12
    assert rel_norm(from_abi(h.field("rho_gnd"), tensor=False), rho.reshape(-1, 12)) < 1e-12
    fp_dev = np.linalg.norm(o.Fp - np.eye(3)) / np.linalg.norm(o.Fp)
    bound = max(10.0 * d_fp / fp_dev, 1e-12)
    e_nye = rel_norm(from_abi(h.field("nye")), o.alpha)
    e_gnd = rel_norm(from_abi(h.field("rho_gnd"), tensor=False), o.rho_gnd)
    print("Fp difference", d_fp, "Fp - I relative size", fp_dev, "field bound", bound,
          "Nye", e_nye, "rho_GND", e_gnd, flush=True)
    # the parity contract's FP64 bar on the Nye and GND fields (1e-10 normwise); the curl
    # differentiates Fp - I, so the bar is also checked against the Fp difference scaled by
    # |Fp| / |Fp - I| (measured 1e-11 to 3e-11 against 7e-11 to 2e-10)
    assert e_nye < min(bound, 1e-10)
    assert e_gnd < min(bound, 1e-10)


def test_cu64_sgcp_at_8cubed_fp64_matches_oracle(lib):
    rves, path = synth.workload("cu64", n_override=8, n_inc_override=50)
    o, h, out = _run_both(lib, rves[0], path, 3)
    for Po, Pg, Fo, Fg in out:
        assert np.max(np.abs(Pg - Po)) <= 1e-10 * np.abs(Po).max()
    _check_gnd_fields(h, o, rves[0])


def test_cu64_at_6cubed_fp64_to_its_rounding_floor_matches_oracle(lib):
    """FP64 at newton_tol 1e-13 and CG 1e-12: the last Newton steps reach the residual's rounding
    floor (about u64 C11, set by the rounding of F), where CG on the noise breaks down or stalls;
    the increment must still end there, through the floor rule, and agree with the oracle."""
    rves, path = synth.workload("cu64", n_override=6, n_inc_override=50)
    o, h, out = _run_both(lib, rves[0], path, 2, newton_tol=1e-13, cg_tol=1e-12)
    for Po, Pg, Fo, Fg in out:
        assert np.max(np.abs(Pg - Po)) <= 1e-10 * np.abs(Po).max()


_MIXED_ORACLE = {}


def _mixed_oracle_p11(rve, path, n_inc):
    """<P>_11 of the oracle at tight tolerances after each of the first n_inc increments
    (computed once per module)."""
    if n_inc not in _MIXED_ORACLE:
        o = solver.RVESolver(rve, newton_tol=1e-11, cg_tol=1e-10)
        out = []
        for k in range(1, n_inc + 1):
            assert o.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)["converged"]
            out.append(o.macro()[0][0])
        _MIXED_ORACLE[n_inc] = out
    return _MIXED_ORACLE[n_inc]


@pytest.mark.parametrize("env", [{}, {"RVE_TANGENT16": "0"}, {"RVE_PLANE": "0"}],
                         ids=["fp16_tangent", "fp32_tangent", "pencil_path"])
def test_cu64_mixed_precision_macro_stress_within_1e4_of_oracle(lib, env, monkeypatch):
    """Mixed form (FP32 spectral path; FP16 or FP32 tangent copy; plane or pencil kernels) at
    its performance tolerances against the FP64 oracle at tight tolerances: <P>_11 within
    1e-4 relative at every increment."""
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    rves, path = synth.workload("cu64", n_override=8, n_inc_override=50)
    ref = _mixed_oracle_p11(rves[0], path, 3)
    h = lib.Homogenizer(rves, precision=lib.RVE_MIXED, newton_tol=1e-6, cg_tol=1e-3, max_cg=3000, max_newton=150)
    worst = 0.0
    for k in range(1, 4):
        print(f"mixed increment {k} {env}", flush=True)
        h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        Pg = h.macro()[0]
        worst = max(worst, abs(Pg[0] - ref[k - 1]) / abs(ref[k - 1]))
    print("worst relative <P>_11 difference", worst, flush=True)
    assert worst <= 1e-4


def test_ragged_grid_fp64_matches_oracle(lib):
    """A 10 x 6 x 12 grid (radix 2, 3, 5 transforms, odd plane sizes) through whole increments."""
    mat = synth.material("Cu", rho0=1e11, c_gnd=1.0)
    rve = synth.voronoi_rve(311, (10, 6, 12), 4, 2e-6, mat)
    path = synth.uniaxial_tension(0.05, 50, 1e-4)
    o, h, out = _run_both(lib, rve, path, 2, newton_tol=1e-13, cg_tol=1e-12)
    for Po, Pg, Fo, Fg in out:
        print("  <P> difference", np.max(np.abs(Pg - Po)) / np.abs(Po).max(), flush=True)
        assert np.max(np.abs(Pg - Po)) <= 1e-10 * np.abs(Po).max()
    _check_gnd_fields(h, o, rve)


@pytest.mark.parametrize("shape", [(8, 8, 8), (12, 9, 10), (6, 5, 4)])
def test_factorised_projection_equals_the_nine_component_form(lib, shape):
    """The CG operator as divergence stencil, three transforms, 1/|k|^2 and gradient stencil
    (projection 0) against the nine-component projection of eq. 17 (projection 1), FP64, two
    whole increments at tight tolerances, on even planes and on planes with an odd row count:
    <P> within 1e-11 and the F field within 1e-11 (the forms differ by rounding only), and the
    timed families show that each form ran."""
    mat = synth.material("Cu", rho0=1e11, c_gnd=1.0)
    rve = synth.voronoi_rve(501, shape, 5, 2e-6, mat)
    path = synth.uniaxial_tension(0.05, 50, 1e-4)
    res = {}
    for form in (0, 1):
        h = lib.Homogenizer([rve], precision=lib.RVE_FP64, newton_tol=1e-13, cg_tol=1e-12, max_cg=4000,
                            projection=form)
        h.timing_start(["cg_grad"])
        Ps = []
        for k in (1, 2):
            print(f"form {form} shape {shape} increment {k}", flush=True)
            st = h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)[0]
            Ps.append(h.macro()[0])
        n_grad = h.timing_read("cg_grad")[0]
        assert (n_grad > 0) == (form == 0), n_grad
        res[form] = (np.array(Ps), from_abi(h.field("F")), st["cg_iters"])
        h.close()
    dP = np.abs(res[0][0] - res[1][0]).max() / np.abs(res[1][0]).max()
    dF = rel_norm(res[0][1], res[1][1])
    print("  <P> difference", dP, "F difference", dF, "cg", res[0][2], res[1][2], flush=True)
    assert dP <= 1e-11
    assert dF <= 1e-11


def test_factorised_projection_mixed_form_matches_fp64(lib):
    """The mixed form with the factorised CG operator on the 16^3 workload at the benchmark
    tolerances: no FP64 fallback and <P>_11 within 1e-4 of the FP64 nine-component form over
    10 increments."""
    rves, path = synth.workload("cu16")
    curves = {}
    for prec, form in ((lib.RVE_MIXED, 0), (lib.RVE_FP64, 1)):
        h = lib.Homogenizer(rves, precision=prec, newton_tol=1e-6, cg_tol=1e-3, max_cg=3000, max_newton=150,
                            projection=form)
        c = []
        for k in range(1, 11):
            st = h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)[0]
            if prec == lib.RVE_MIXED:
                assert st["fp64_fallback"] == 0, (k, st)
            c.append(h.macro()[0][0])
        h.close()
        curves[prec] = np.array(c)
    diff = np.abs(curves[lib.RVE_MIXED] - curves[lib.RVE_FP64]) / np.abs(curves[lib.RVE_FP64]).max()
    print("largest relative <P>_11 difference", diff.max(), flush=True)
    assert diff.max() <= 1e-4


def test_adjoint_solve_matches_oracle_transposed_cg(lib):
    """rve_adjoint_solve after three increments of the 64-grain SGCP workload at 6^3 (FP64):
    lam from G(K^T : lam) = G(g) against the oracle's conjugate gradients with its own tangent
    (central differences) at the same converged state (measured 2e-7 apart; bar 1e-5).  The
    untransposed system's solution differs by more than 2e-3, which the test checks, so a plain
    K : lam fails it."""
    rves, path = synth.workload("cu64", n_override=6, n_inc_override=50)
    rve = rves[0]
    h = lib.Homogenizer([rve], precision=lib.RVE_FP64, newton_tol=1e-13, cg_tol=1e-12, max_cg=4000)
    o = solver.RVESolver(rve, newton_tol=1e-13, cg_tol=1e-12)
    for k in range(1, 4):
        if k == 3:
            Fp_n, rs_n, rg_n = o.Fp.copy(), o.rho_ssd.copy(), o.rho_gnd.copy()
        assert o.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)["converged"]
        h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
    K = constitutive.tangent_fd(o.model, o.gid, o.F, Fp_n, rs_n, rg_n, path.dt, o.dg)
    g = np.random.default_rng(5).standard_normal((rve.n_vox, 3, 3))
    lam_o, _ = solver.adjoint_solve(o.project, K, g, path.mask, 1e-12, 4000)
    lam_k, _ = solver.conjugate_gradient(lambda y: o.project(np.einsum("vijkl,vkl->vij", K, y), path.mask),
                                         o.project(g, path.mask), 1e-12, 4000)
    gt = cuda(to_abi(g))
    lt = gt.clone()
    print("adjoint solve 6^3 after 3 increments", flush=True)
    it = h.adjoint_solve(gt, path.mask, lt)
    lam_g = from_abi(lt.cpu().numpy())
    err, sep = rel_norm(lam_g, lam_o), rel_norm(lam_k, lam_o)
    print("adjoint: cg", it, "gpu vs oracle", err, "K vs K^T solutions", sep, flush=True)
    assert sep > 2e-3
    assert err < 1e-5


def test_adjoint_gradient_of_the_macro_stress_matches_oracle_differences(lib):
    """The adjoint pieces compose into the derivative of one increment's macroscopic stress.
    With L = <P>_11 at the end of increment 3 (64-grain SGCP workload at 6^3, FP64) and
    theta = c_GND: the perturbed equilibrium is G(K : dF + p) = 0 with dF in the range of G and
    p = dP/dtheta at fixed F, and G is an orthogonal projection, so dL/dtheta = <e - lam, p>
    with G(K^T : lam) = G(K^T : e), e the unit 11 field.  p comes from rve_stress_sensitivity
    chained through eq. 7, lam from rve_adjoint_solve, K^T : e from rve_constitutive_batch.
    Against central differences of the oracle's whole increment in c_GND (from the oracle's own
    state after two increments; steps of 1e-2 and 1e-3 agree to 3e-7).  Without lam the value
    is off by more than 1e-2, which the test checks."""
    import copy
    import dataclasses
    import torch
    rves, path = synth.workload("cu64", n_override=6, n_inc_override=50)
    rve = rves[0]
    mat = rve.material
    V = rve.n_vox
    o = solver.RVESolver(rve, newton_tol=1e-13, cg_tol=1e-12)
    for k in (1, 2):
        assert o.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)["converged"]

    def L_of(c):
        o2 = copy.deepcopy(o)
        o2.model.mat = dataclasses.replace(o2.model.mat, c_gnd=c)
        assert o2.step(path.F_bar[3], path.mask, path.P_bar[3], path.dt)["converged"]
        return o2.macro()[0].reshape(-1)[0]

    eps = 1e-3 * mat.c_gnd
    dL_ref = (L_of(mat.c_gnd + eps) - L_of(mat.c_gnd - eps)) / (2 * eps)

    h = lib.Homogenizer([rve], precision=lib.RVE_FP64, newton_tol=1e-13, cg_tol=1e-12, max_cg=4000)
    for k in (1, 2):
        h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
    start = {n: h.field(n) for n in ("Fp", "rho_ssd", "rho_gnd")}
    print("adjoint gradient: increment 3", flush=True)
    h.step(path.F_bar[3], path.mask, path.P_bar[3], path.dt)
    F_end, dg_end = h.field("F"), h.field("dg")
    gid = cuda(rve.grain_of_voxel.reshape(-1))
    args = [cuda(F_end), cuda(start["Fp"]), cuda(start["rho_ssd"]), cuda(start["rho_gnd"]), path.dt]
    # K at the converged point (sample frame), then g = K^T : e, g_kl = K_11kl
    t_dg = cuda(dg_end)
    t_P = torch.zeros((9, V), dtype=torch.float64, device="cuda:0")
    t_K = torch.zeros((81, V), dtype=torch.float64, device="cuda:0")
    lib.constitutive_batch(mat, rve.quats, gid, *args, t_dg, t_P, t_K)
    g = t_K[0:9].clone()
    lam = torch.zeros_like(g)
    it = h.adjoint_solve(g, path.mask, lam)
    # p = dP/dc_GND at fixed F: dP/dtau_c times d tau_c,a / dc = (mu b)^2 sum_b q_ab rho_GND,b / (2 tau_c,a)
    t_S = torch.zeros((108, V), dtype=torch.float64, device="cuda:0")
    lib.stress_sensitivity(mat, rve.quats, gid, *args, cuda(dg_end), t_S)
    torch.cuda.synchronize()
    dPdtc = t_S.cpu().numpy().reshape(12, 9, V)
    model = constitutive.MaterialModel(mat, rve.quats)
    forest = start["rho_ssd"] + mat.c_gnd * start["rho_gnd"]
    mub = model.mu * mat.burgers
    tau_c = mub * np.sqrt(model.q @ forest)                          # (12, V)
    dtc = mub * mub * (model.q @ start["rho_gnd"]) / (2.0 * tau_c)   # (12, V)
    p = np.einsum("arv,av->rv", dPdtc, dtc)                          # (9, V)
    lam_h = lam.cpu().numpy()
    dL = float(np.mean(p[0] - np.sum(lam_h * p, axis=0)))
    dL_local = float(np.mean(p[0]))
    err = abs(dL - dL_ref) / abs(dL_ref)
    print("adjoint gradient", dL, "oracle differences", dL_ref, "relative", err, "cg", it,
          "without lam", dL_local, flush=True)
    assert abs(dL_local - dL_ref) > 1e-2 * abs(dL_ref)
    assert err < 1e-4


def test_adjoint_solve_rejects_a_mixed_handle_and_an_unstepped_rve(lib):
    rves, path = synth.workload("cu16", n_override=8, n_inc_override=20)
    g = cuda(np.zeros((9, rves[0].n_vox)))
    h = lib.Homogenizer(rves, precision=lib.RVE_FP64)
    with pytest.raises(lib.RVEError):
        h.adjoint_solve(g, path.mask, g.clone())          # no increment taken yet
    hm = lib.Homogenizer(rves, precision=lib.RVE_MIXED)
    hm.step(path.F_bar[1], path.mask, path.P_bar[1], path.dt)
    with pytest.raises(lib.RVEError):
        hm.adjoint_solve(g, path.mask, g.clone())         # needs an FP64 handle


def test_save_load_replays_an_increment_bit_exactly(lib):
    rves, path = synth.workload("cu16", n_override=8, n_inc_override=20)
    h = lib.Homogenizer(rves, precision=lib.RVE_FP64, newton_tol=1e-10, cg_tol=1e-8)
    for k in (1, 2):
        h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
    state = h.save_state()
    h.step(path.F_bar[3], path.mask, path.P_bar[3], path.dt)
    first = {n: h.field(n) for n in ("F", "P", "Fp", "rho_ssd", "rho_gnd", "nye", "dg")}
    P_first = h.macro()[0]
    h.load_state(state)
    P_loaded = h.macro()[0]
    h.step(path.F_bar[3], path.mask, path.P_bar[3], path.dt)
    for n, a in first.items():
        assert np.array_equal(h.field(n), a), n
    assert np.array_equal(h.macro()[0], P_first)
    assert not np.array_equal(P_loaded, P_first)


def test_failed_increment_leaves_state_unchanged(lib):
    rves, path = synth.workload("cu16", n_override=8, n_inc_override=20)
    h = lib.Homogenizer(rves, precision=lib.RVE_FP64, newton_tol=1e-10, cg_tol=1e-8)
    h.step(path.F_bar[1], path.mask, path.P_bar[1], path.dt)
    before = {n: h.field(n) for n in ("F", "P", "Fp", "rho_ssd", "rho_gnd", "nye", "dg")}
    P_before = h.macro()[0]
    # one Newton iteration and no line search cannot meet a 1e-15 tolerance
    h2 = lib.Homogenizer(rves, precision=lib.RVE_FP64, newton_tol=1e-15, cg_tol=1e-8, max_newton=1,
                         max_backtrack=0)
    h2.load_state(h.save_state())
    with pytest.raises(lib.RVEError) as e:
        h2.step(path.F_bar[2], path.mask, path.P_bar[2], path.dt)
    assert e.value.code == -4 and e.value.stats[0]["status"] == -4
    for n, a in before.items():
        assert np.array_equal(h2.field(n), a), n
    assert np.array_equal(h2.macro()[0], P_before)


def test_batch_of_uneven_rves_equals_separate_handles(lib):
    mat = synth.material("Cu", rho0=1e11, c_gnd=1.0)
    a = synth.voronoi_rve(401, (8, 8, 8), 5, 3e-6, mat)
    b = synth.voronoi_rve(402, (6, 10, 4), 3, 2e-6, synth.material("Ni", rho0=1e11, c_gnd=1.0))
    path = synth.uniaxial_tension(0.05, 50, 1e-4)
    hb = lib.Homogenizer([a, b], precision=lib.RVE_FP64, newton_tol=1e-10, cg_tol=1e-8)
    ha = lib.Homogenizer([a], precision=lib.RVE_FP64, newton_tol=1e-10, cg_tol=1e-8)
    hs = lib.Homogenizer([b], precision=lib.RVE_FP64, newton_tol=1e-10, cg_tol=1e-8)
    for k in (1, 2):
        hb.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        ha.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        hs.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        assert np.array_equal(hb.macro(0)[0], ha.macro(0)[0])
        assert np.array_equal(hb.macro(1)[0], hs.macro(0)[0])
    assert np.array_equal(hb.field("rho_gnd", 1), hs.field("rho_gnd", 0))


def test_nye_gnd_returns_the_committed_fields(lib):
    """rve_nye_gnd hands out the Nye tensor and GND densities that the last increment committed
    (the same values as the field reader), for each RVE of a batch."""
    mat = synth.material("Cu", rho0=1e11, c_gnd=1.0)
    rves = [synth.voronoi_rve(700 + i, (8, 8, 8), 4, 2e-6, mat) for i in range(2)]
    path = synth.uniaxial_tension(0.05, 50, 1e-4)
    h = lib.Homogenizer(rves, precision=lib.RVE_FP64, newton_tol=1e-10, cg_tol=1e-8)
    for k in (1, 2):
        h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
    for i in range(2):
        nye, rho = h.nye_gnd(i)
        assert np.array_equal(nye, h.field("nye", i))
        assert np.array_equal(rho, h.field("rho_gnd", i))
        assert np.abs(nye).max() > 0 and rho.max() > 0
    with pytest.raises(lib.RVEError):
        lib.check(lib.lib().rve_nye_gnd(h.h, 2, None, None))
    h.close()


def test_mixed_batch_with_graphs_on_concurrent_workers(lib):
    """Sixteen mixed-form RVEs on eight host workers with CG graphs: every RVE's first increment
    (when each worker captures its graphs while others start their solves) and the next one
    succeed, and the result equals the same handle driven by one worker without graphs."""
    mat = synth.material("Cu", rho0=1e11, c_gnd=1.0)
    rves = [synth.voronoi_rve(600 + i, (16, 16, 16), 6, 2e-6, mat) for i in range(16)]
    path = synth.uniaxial_tension(0.05, 50, 1e-4)
    out = {}
    for workers, graph in ((8, 1), (1, 0)):
        h = lib.Homogenizer(rves, precision=lib.RVE_MIXED, newton_tol=1e-6, cg_tol=1e-3, use_graph=graph,
                            workers=workers)
        for k in (1, 2):
            st = h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
            assert all(s["status"] == 0 and s["fp64_fallback"] == 0 for s in st)
        out[workers] = np.array([h.macro(i)[0] for i in range(len(rves))])
        h.close()
    assert np.array_equal(out[8], out[1])


def test_kernel_timing_counts_live_launches(lib):
    rves, path = synth.workload("cu16", n_override=8, n_inc_override=20)
    h = lib.Homogenizer(rves, precision=lib.RVE_MIXED, newton_tol=1e-6, cg_tol=1e-3)
    h.step(path.F_bar[1], path.mask, path.P_bar[1], path.dt)
    h.timing_start(["cg_prep", "mid", "mid3", "slip_fast"])
    st = h.step(path.F_bar[2], path.mask, path.P_bar[2], path.dt)[0]
    n_prep, ms_prep, b_prep = h.timing_read("cg_prep")
    n_mid, ms_mid, b_mid = h.timing_read("mid")
    n_mid3, ms_mid3, b_mid3 = h.timing_read("mid3")
    n_fast, _, vox = h.timing_read("slip_fast")
    assert n_fast >= 1 and vox == n_fast * rves[0].n_vox
    # every CG iteration applies the operator once, in the factorised form (three components in
    # the z pass); each residual evaluation takes one nine-component z pass
    assert n_mid3 == st["cg_iters"] and n_mid == st["residual_evals"]
    assert st["cg_iters"] <= n_prep <= st["cg_iters"] + st["newton_iters"]
    assert ms_mid > 0 and b_mid == n_mid * 2 * 9 * 2 * 4 * 5 * 8 * 8
    assert ms_mid3 > 0 and b_mid3 == n_mid3 * 2 * 3 * 2 * 4 * 5 * 8 * 8
    assert h.timing_read("plane_fwd")[0] == 0          # not selected
    h.timing_start([])
    with pytest.raises(lib.RVEError):
        lib.check(lib.lib().rve_timing_start(h.h, 1 << 11))       # unknown family bit


def test_cu64_mixed_runs_the_whole_path_in_fp32_within_1e4_of_the_fp64_form(lib):
    """The 64^3 strain-gradient workload through all 50 increments (5 % strain) in the mixed
    form at the benchmark tolerances: no increment falls back to the FP64 spectral path, and
    <P>_11 stays within 1e-4 (relative to the largest stress of the curve) of the FP64 form at
    the same tolerances at every increment."""
    rves, path = synth.workload("cu64")
    curves = {}
    for prec in (lib.RVE_MIXED, lib.RVE_FP64):
        h = lib.Homogenizer(rves, precision=prec, newton_tol=1e-6, cg_tol=1e-3, max_cg=3000, max_newton=150)
        c = []
        for k in range(1, path.n_inc + 1):
            st = h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)[0]
            if prec == lib.RVE_MIXED:
                assert st["fp64_fallback"] == 0, (k, st)
                assert st["discarded_voxel_iterations"] == 0, (k, st)
            c.append(h.macro()[0][0])
        h.close()
        curves[prec] = np.array(c)
        print(f"precision {prec}: <P>_11 at 5 % {c[-1]:.6e}", flush=True)
    ref = curves[lib.RVE_FP64]
    diff = np.abs(curves[lib.RVE_MIXED] - ref) / np.abs(ref).max()
    print("largest relative <P>_11 difference, mixed vs FP64", diff.max(), flush=True)
    assert diff.max() <= 1e-4


def test_adjoint_solve_refuses_a_tangent_that_is_not_the_committed_increments(lib):
    """After rve_load_state, and after an increment that failed, the stored tangent belongs to
    another state than the last committed increment: rve_adjoint_solve refuses until an
    increment has been taken again."""
    rves, path = synth.workload("cu16", n_override=8, n_inc_override=20)
    V = rves[0].n_vox
    g = cuda(np.zeros((9, V)))
    h = lib.Homogenizer(rves, precision=lib.RVE_FP64, newton_tol=1e-10, cg_tol=1e-8)
    h.step(path.F_bar[1], path.mask, path.P_bar[1], path.dt)
    state = h.save_state()
    h.step(path.F_bar[2], path.mask, path.P_bar[2], path.dt)
    h.adjoint_solve(g, path.mask, g.clone())                # valid: the tangent of increment 2
    h.load_state(state)
    with pytest.raises(lib.RVEError):
        h.adjoint_solve(g, path.mask, g.clone())
    h.step(path.F_bar[2], path.mask, path.P_bar[2], path.dt)
    h.adjoint_solve(g, path.mask, g.clone())
    h2 = lib.Homogenizer(rves, precision=lib.RVE_FP64, newton_tol=1e-15, cg_tol=1e-8, max_newton=1,
                         max_backtrack=0)
    h2.load_state(state)
    with pytest.raises(lib.RVEError):
        h2.step(path.F_bar[2], path.mask, path.P_bar[2], path.dt)   # fails (RVE_ENOCONV)
    with pytest.raises(lib.RVEError):
        h2.adjoint_solve(g, path.mask, g.clone())


def test_lognormal_grains_on_a_radix_3_and_5_grid_fp64_match_oracle(lib):
    """The paper's kind of microstructure (equiaxed grains with lognormal sizes, Section 2.2)
    on a 15^3 = 3 x 5 grid (radix-3 and radix-5 transforms on every axis), two increments of
    the strain-gradient Cu workload in FP64: <P> to the 1e-10 bar, and the Nye and GND fields."""
    gid, _, _ = synth.lognormal_grains(21, (15, 15, 15), 12)
    quats = synth.shoemake_quaternions(synth.SplitMix64(1021), 12)
    mat = synth.material("Cu", rho0=1e11, c_gnd=1.0)
    rve = synth.RVE(n=(15, 15, 15), voxel_size=1.5e-6, grain_of_voxel=gid, quats=quats, material=mat, seed=21)
    path = synth.uniaxial_tension(0.05, 50, 1e-4)
    o, h, out = _run_both(lib, rve, path, 2, newton_tol=1e-12, cg_tol=1e-11)
    for Po, Pg, Fo, Fg in out:
        print("  <P> difference", np.max(np.abs(Pg - Po)) / np.abs(Po).max(), flush=True)
        assert np.max(np.abs(Pg - Po)) <= 1e-10 * np.abs(Po).max()
    _check_gnd_fields(h, o, rve)


@pytest.mark.parametrize("load", ["shear", "biaxial", "stress_shear"])
def test_general_mixed_control_fp64_matches_oracle(lib, load):
    """Mixed control beyond uniaxial tension (eq. 15 and the zero-frequency rule): simple shear
    (normal stresses free), equibiaxial tension (P_33 free) and a stress-controlled shear (a
    prescribed nonzero P_12 with F_12 free), two increments of the strain-gradient Cu workload
    at 8^3 in FP64 against the oracle: <P> and <F> to the 1e-10 bar, and the prescribed
    averages met."""
    rves, _ = synth.workload("cu64", n_override=8)
    path = {"shear": lambda: synth.simple_shear(0.01, 10, 1e-4),
            "biaxial": lambda: synth.biaxial_tension(0.005, 10, 1e-4),
            "stress_shear": lambda: synth.stress_controlled_shear(20e6, 10, 10.0)}[load]()
    o, h, out = _run_both(lib, rves[0], path, 2)
    for k, (Po, Pg, Fo, Fg) in enumerate(out, start=1):
        scale = np.abs(Po).max()
        print(f"  {load} increment {k}: <P> difference {np.max(np.abs(Pg - Po)) / scale:.2e}", flush=True)
        assert np.max(np.abs(Pg - Po)) <= 1e-10 * scale
        assert np.max(np.abs(Fg - Fo)) <= 1e-11
        free = path.mask == 0
        assert np.max(np.abs(Pg[free] - path.P_bar[k][free])) <= 1e-8 * scale
        fixed = path.mask == 1
        assert np.max(np.abs(Fg[fixed] - path.F_bar[k][fixed])) <= 1e-12


def test_time_step_cutback_equals_explicit_half_increments(lib):
    """With max_cutbacks, an increment that fails is committed as two increments of half the
    time step (targets at the midpoint, then at the end).  Here the Newton iteration budget is
    set to what each half needs, so that a double-size increment fails directly; with one level
    of cut-back the handle commits it in two halves, bit-identical to two explicit increments."""
    rves, path = synth.workload("cu16", n_override=8, n_inc_override=20)
    opts = dict(precision=lib.RVE_FP64, newton_tol=1e-10, cg_tol=1e-8, max_continuation=1)
    b = lib.Homogenizer(rves, max_newton=40, **opts)
    need = 0
    # the midpoint target exactly as the library forms it: (previous target + target) / 2
    F_mid = 0.5 * (path.F_bar[0] + path.F_bar[2])
    P_mid = 0.5 * (path.P_bar[0] + path.P_bar[2])
    for F_t, P_t in ((F_mid, P_mid), (path.F_bar[2], path.P_bar[2])):
        need = max(need, b.step(F_t, path.mask, P_t, path.dt)[0]["newton_iters"])
    ref = {n: b.field(n) for n in ("F", "P", "Fp", "rho_ssd", "rho_gnd", "dg")}
    P_ref = b.macro()[0]
    print("Newton iterations of the larger half", need, flush=True)
    plain = lib.Homogenizer(rves, max_newton=need, **opts)
    with pytest.raises(lib.RVEError):
        plain.step(path.F_bar[2], path.mask, path.P_bar[2], 2 * path.dt)
    a = lib.Homogenizer(rves, max_newton=need, max_cutbacks=1, **opts)
    st = a.step(path.F_bar[2], path.mask, path.P_bar[2], 2 * path.dt)[0]
    print("cut-back stats", st, flush=True)
    assert st["cutbacks"] == 1 and st["status"] == 0
    assert st["discarded_voxel_iterations"] > 0
    for n, v in ref.items():
        assert np.array_equal(a.field(n), v), n
    assert np.array_equal(a.macro()[0], P_ref)


def test_cu16_whole_curve_matches_the_oracle_reference():
    """The 16^3 FP64 workload (8 grains, Cu, tau0 = 10 MPa, no gradient term) through all 20
    increments to 1 %: <P> and <F> after every increment against the oracle's curve stored in
    tests/golden/c1_cu16_curve.json (written by tests/golden/make_c1_curve.py, which calls only
    the oracle, at the same tolerances): the 1e-10 bar at every increment."""
    import json
    import os
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_01946_amd as m
    m.lib()
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_cu16_curve.json")) as f:
        ref = json.load(f)
    rves, path = synth.workload("cu16")
    h = m.Homogenizer(rves, precision=m.RVE_FP64, newton_tol=ref["newton_tol"], cg_tol=ref["cg_tol"],
                      max_cg=20000, max_newton=80)
    worst = 0.0
    scale = np.abs(np.array(ref["P_avg"])).max()
    for k in range(1, path.n_inc + 1):
        h.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
        Pg, Fg, _ = h.macro()
        d = np.max(np.abs(Pg - np.array(ref["P_avg"][k - 1]))) / scale
        worst = max(worst, d)
        print(f"increment {k}: <P>_11 {Pg[0]:.10e} reference {ref['P_avg'][k - 1][0]:.10e} difference {d:.2e}",
              flush=True)
        assert d <= 1e-10
        assert np.max(np.abs(Fg - np.array(ref["F_avg"][k - 1]))) <= 1e-12
    print("largest difference over the curve", worst, flush=True)
