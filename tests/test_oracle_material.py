"""Pins of the oracle's material point (Section 2.1, eqs. 1-9, 14)."""
import numpy as np

import synth
from oracle import constitutive as cst
from oracle import elasticity, reference


def _setup(V=12, amp=3e-4, seed=3, c_gnd=1.0):
    mat = synth.material("Cu", tau0=10e6, c_gnd=c_gnd)
    q = synth.shoemake_quaternions(synth.SplitMix64(seed), 4)
    model = cst.MaterialModel(mat, q)
    gid = np.arange(V) % 4
    F = synth.random_deformations(seed + 1, V, amp).reshape(V, 3, 3)
    Fp_n = synth.random_deformations(seed + 2, V, 2e-4).reshape(V, 3, 3)
    rs = model.rho0 * (1 + synth.random_field(seed + 3, (V, 12), 0, 1))
    rg = synth.random_field(seed + 4, (V, 12), 0, 1) * 1e12
    return mat, model, gid, F, Fp_n, rs, rg


def test_elastic_limit_is_st_venant_kirchhoff():
    """tau0 -> huge: no slip, Fp = Fp_n = I, and eq. 14 reduces to P = F (C : E)."""
    mat = synth.material("Al", tau0=1e14, c_gnd=0.0)
    q = synth.shoemake_quaternions(synth.SplitMix64(4), 3)
    model = cst.MaterialModel(mat, q)
    V = 9
    F = synth.random_deformations(5, V, 5e-3).reshape(V, 3, 3)
    gid = np.arange(V) % 3
    out = cst.update(model, gid, F, np.tile(np.eye(3), (V, 1, 1)), np.full((V, 12), model.rho0),
                     np.zeros((V, 12)), 1.0, np.zeros((V, 12)))
    P_ref = reference.svk_stress(F, model.C[gid])
    assert np.allclose(out["P"], P_ref, rtol=1e-12, atol=1e-6)
    assert np.abs(out["dg"]).max() < 1e-100


def test_converged_slip_solves_flow_rule_and_shares_root():
    mat, model, gid, F, Fp_n, rs, rg = _setup()
    dt = 0.5
    out = cst.update(model, gid, F, Fp_n, rs, rg, dt, np.zeros_like(rs))
    assert out["converged"].all()
    pd = cst.PointData(model, gid, Fp_n, rs, rg)
    R = cst.residual(pd, F, out["dg"], dt)
    assert np.all(np.abs(R).max(axis=1) <= 1e-10 * np.abs(out["dg"]).max(axis=1))
    # flow rule written out independently from the stress of the returned state
    tau = np.einsum("vij,vaij->va", out["S"], model.P0[gid])
    g = dt * mat.gamma0_dot * (np.abs(tau) / out["tau_c"]) ** (1 / mat.m_rate) * np.sign(tau)
    assert np.allclose(g, out["dg"], rtol=1e-8, atol=1e-18)
    # a different starting point reaches the same root
    out2 = cst.update(model, gid, F, Fp_n, rs, rg, dt, 1e-4 * np.ones_like(rs))
    assert np.allclose(out2["dg"], out["dg"], rtol=1e-9, atol=1e-16)
    assert np.allclose(out2["P"], out["P"], rtol=1e-11)


def test_state_update_formulas():
    """Fp = (I + sum dg s(x)m) Fp_n (eq. 2, backward Euler); Fe = F Fp^-1; rho_SSD by eq. 8
    integrated over the increment with the mean free path frozen;
    tau_c by eq. 7 with the forest densities; P from S by eq. 14."""
    mat, model, gid, F, Fp_n, rs, rg = _setup()
    out = cst.update(model, gid, F, Fp_n, rs, rg, 0.5, np.zeros_like(rs))
    s0, m0 = __import__("oracle.tables", fromlist=["x"]).slip_systems()
    R = model.R[gid]
    s = np.einsum("vij,aj->vai", R, s0)
    m = np.einsum("vij,aj->vai", R, m0)
    L = np.einsum("va,vai,vaj->vij", out["dg"], s, m)
    assert np.allclose(out["Fp"], (np.eye(3) + L) @ Fp_n, rtol=1e-14)
    Fe = F @ np.linalg.inv(out["Fp"])
    assert np.allclose(out["P"], Fe @ out["S"] @ np.linalg.inv(out["Fp"]).transpose(0, 2, 1), rtol=1e-10)
    q = model.q
    forest = rs + mat.c_gnd * rg
    ell = mat.K_sim / np.sqrt(forest.sum(1, keepdims=True) - forest)
    # eq. 8 over the increment with l frozen: rho_n exp(-x) + u (1 - exp(-x)) / (x b l)
    u = np.abs(out["dg"])
    x = 2 * mat.y_c * u / mat.burgers
    rho_new = rs * np.exp(-x) + np.where(x > 0, u * (1 - np.exp(-x)) / np.where(x > 0, x, 1), u) / (mat.burgers * ell)
    assert np.allclose(out["rho_ssd"], rho_new, rtol=1e-12)
    mu = elasticity.slip_plane_shear_modulus(mat.C11, mat.C12, mat.C44)
    assert np.allclose(out["tau_c"], mu * mat.burgers * np.sqrt(forest @ q.T), rtol=1e-14)


def test_fd_tangent_step_consistency():
    mat, model, gid, F, Fp_n, rs, rg = _setup(V=4)
    dt = 0.5
    out = cst.update(model, gid, F, Fp_n, rs, rg, dt, np.zeros_like(rs))
    K1 = cst.tangent_fd(model, gid, F, Fp_n, rs, rg, dt, out["dg"], step=1e-8)
    K2 = cst.tangent_fd(model, gid, F, Fp_n, rs, rg, dt, out["dg"], step=4e-8)
    assert np.abs(K1 - K2).max() / np.abs(K1).max() < 1e-5


def test_schmid_single_crystal_steady_flow():
    """[100] single crystal, hardening off: 8 systems with Schmid factor 1/sqrt(6) carry the
    plastic strain rate, so steady flow has S_xx = (tau0/M) (rate / (8 M gdot0))^m
    (23.087 MPa for tau0 = 10 MPa, rate = gdot0 = 1e-3/s)."""
    mat = synth.material("Cu", tau0=10e6, c_gnd=0.0, hardening=0)
    path = synth.uniaxial_tension(0.01, 20, 1e-3)
    res = reference.material_point_path(mat, [1, 0, 0, 0], path)
    M = 1 / np.sqrt(6)
    expect = (10e6 / M) * (1e-3 / (8 * M * 1e-3)) ** 0.05
    assert abs(expect / 23.087e6 - 1) < 1e-4
    S_last = res[-1][2]
    assert abs(S_last[0, 0] / expect - 1) < 1.5e-3
    tau = np.abs(res[-1][3])
    assert np.sum(tau > 0.9 * tau.max()) == 8
    # the lateral stresses vanish
    assert abs(res[-1][1][1, 1]) < 1e-3 and abs(res[-1][1][2, 2]) < 1e-3


def test_fd_gnd_sensitivity_step_consistency_and_zero_gradient_term():
    """dP/d rho_GND by central differences: two steps agree (the difference quotient has
    converged), and with c_GND = 0 the GND densities do not reach the stress at all."""
    mat, model, gid, F, Fp_n, rs, rg = _setup(V=4)
    dt = 0.5
    out = cst.update(model, gid, F, Fp_n, rs, rg, dt, np.zeros_like(rs))
    S1 = cst.stress_gnd_sensitivity_fd(model, gid, F, Fp_n, rs, rg, dt, out["dg"], rel_step=1e-4)
    S2 = cst.stress_gnd_sensitivity_fd(model, gid, F, Fp_n, rs, rg, dt, out["dg"], rel_step=4e-4)
    assert np.abs(S1).max() > 0
    assert np.abs(S1 - S2).max() / np.abs(S1).max() < 2e-6
    mat0, model0, *_ = _setup(V=4, c_gnd=0.0)
    out0 = cst.update(model0, gid, F, Fp_n, rs, rg, dt, np.zeros_like(rs))
    S0 = cst.stress_gnd_sensitivity_fd(model0, gid, F, Fp_n, rs, rg, dt, out0["dg"])
    assert not S0.any()


def test_fd_density_parameter_sensitivity():
    """d rho_SSD / d(K, y_c) of eq. 8 by central differences: y_c enters linearly, so two steps
    agree to rounding; the K quotient has converged; without hardening both vanish exactly."""
    mat, model, gid, F, Fp_n, rs, rg = _setup(V=6)
    dt = 0.5
    out = cst.update(model, gid, F, Fp_n, rs, rg, dt, np.zeros_like(rs))
    S1 = cst.density_param_sensitivity_fd(model, gid, Fp_n, rs, rg, out["dg"], rel_step=1e-4)
    S2 = cst.density_param_sensitivity_fd(model, gid, Fp_n, rs, rg, out["dg"], rel_step=4e-4)
    for row, bar in ((0, 1e-6), (1, 1e-9)):
        assert np.abs(S1[:, row]).max() > 0
        assert np.abs(S1[:, row] - S2[:, row]).max() <= bar * np.abs(S1[:, row]).max()
    # no slip on a system, no change of its density with either parameter
    dg = out["dg"].copy()
    dg[:, 3] = 0.0
    S3 = cst.density_param_sensitivity_fd(model, gid, Fp_n, rs, rg, dg)
    assert not S3[:, :, 3].any()
    mat0 = synth.material("Cu", tau0=10e6, c_gnd=1.0, hardening=0)
    model0 = cst.MaterialModel(mat0, synth.shoemake_quaternions(synth.SplitMix64(3), 4))
    assert not cst.density_param_sensitivity_fd(model0, gid, Fp_n, rs, rg, out["dg"]).any()


def test_fd_fp_sensitivity_step_consistency_and_tangent_identity():
    """dP/dFp_n along random directions by central differences: the quotient has converged,
    and it satisfies dP = -K : (Fe0 dFp_n) - P dFp_n^T Fp_n^-T with the oracle's own
    difference tangent K (the slip increments depend on F and Fp_n only through
    Fe0 = F Fp_n^-1, and P = Phi(Fe0) Fp_n^-T)."""
    mat, model, gid, F, Fp_n, rs, rg = _setup(V=6, amp=2e-3)
    dt = 0.5
    out = cst.update(model, gid, F, Fp_n, rs, rg, dt, np.zeros_like(rs))
    D = synth.random_field(31, (6, 3, 3))
    S1 = cst.stress_fp_direction_fd(model, gid, F, Fp_n, rs, rg, dt, out["dg"], D, step=1e-7)
    S2 = cst.stress_fp_direction_fd(model, gid, F, Fp_n, rs, rg, dt, out["dg"], D, step=4e-7)
    assert np.abs(S1 - S2).max() <= 1e-5 * np.abs(S1).max()
    K = cst.tangent_fd(model, gid, F, Fp_n, rs, rg, dt, out["dg"])
    Gn = np.linalg.inv(Fp_n)
    Fe0 = F @ Gn
    pred = -np.einsum("vijkl,vkl->vij", K, Fe0 @ D) - out["P"] @ np.swapaxes(D, 1, 2) @ np.swapaxes(Gn, 1, 2)
    assert np.abs(pred - S1).max() <= 1e-5 * np.abs(S1).max()


def _uniform_point(model, rho_ssd, rho_gnd=0.0):
    """One voxel whose twelve systems carry the same densities."""
    return cst.PointData(model, np.zeros(1, dtype=np.int64), np.eye(3)[None],
                         np.full((1, 12), float(rho_ssd)), np.full((1, 12), float(rho_gnd)))


def test_density_update_saturates_at_the_closed_form_fixed_point():
    """Eqs. 8-9 with all twelve systems slipping equally and no GND term: the mean free path
    is K / sqrt(11 rho) (the forest of eq. 9 excludes the system itself), so the SSD density
    stops growing where sqrt(11 rho) / K = 2 y_c rho, i.e. at rho_sat = 11 / (4 y_c^2 K^2)
    (3.40e14 1/m^2 for Cu).  Along the way u = sqrt(rho) obeys du/dgamma = (sqrt(11)/K -
    2 y_c u) / (2 b), so rho(gamma) = (u_sat - (u_sat - u_0) exp(-y_c gamma / b))^2.  A forest
    that included the system itself (12), a dropped factor 2 or 1/b, or K on the wrong side
    each moves the fixed point or the rate."""
    mat = synth.material("Cu", rho0=1e11, c_gnd=0.0)
    model = cst.MaterialModel(mat, [[1.0, 0.0, 0.0, 0.0]])
    b, yc, K = mat.burgers, mat.y_c, mat.K_sim
    rho_sat = 11.0 / (4.0 * yc ** 2 * K ** 2)
    assert abs(rho_sat / 3.395e14 - 1) < 1e-3
    # at the fixed point the density does not move, whatever the slip
    pd = _uniform_point(model, rho_sat)
    assert np.abs(pd.h_ssd).max() * rho_sat ** -0.5 < 1e-12 * np.sqrt(11.0) / K
    out = cst._rho_ssd(pd, np.full((1, 12), 0.3))
    assert np.allclose(out, rho_sat, rtol=1e-12)
    # eq. 7 at a uniform forest: tau_c = mu b sqrt(1.975 rho) (Table 1's row sum)
    mu = elasticity.slip_plane_shear_modulus(mat.C11, mat.C12, mat.C44)
    assert np.allclose(cst._tau_c(pd), mu * b * np.sqrt(1.975 * rho_sat), rtol=1e-13)
    # explicit steps of equal slip follow the closed-form saturation curve
    dgam = 1e-5
    rho = 1e11
    u_sat, u0 = np.sqrt(rho_sat), np.sqrt(1e11)
    checkpoints = (2000, 8000, 40000)
    for n in range(1, checkpoints[-1] + 1):
        rho = float(cst._rho_ssd(_uniform_point(model, rho), np.full((1, 12), dgam))[0, 0])
        if n in checkpoints:
            exact = (u_sat - (u_sat - u0) * np.exp(-yc * n * dgam / b)) ** 2
            # first-order steps: error of order y_c dgamma / b relative
            assert abs(rho / exact - 1) < 2e-3, (n, rho, exact)
    assert abs(rho / rho_sat - 1) < 1e-4


def test_density_step_equals_fine_integration_with_frozen_mean_free_path():
    """Over one increment the mean free path (eq. 9) is held at its start value, and eq. 8 is
    then a linear ODE in the slip; the update must equal its fine-step numerical integration
    (classical Runge-Kutta, 20000 steps) from small slips, where it is the forward-Euler step
    to first order, to slips of 2 y_c |dg| / b up to 40 (aluminium: y_c / b near 200), where
    the forward-Euler step would be negative.  A dropped factor 2, y_c on the wrong side or
    the saturation density from the wrong forest each move the result."""
    for name in ("Cu", "Al"):
        mat = synth.material(name, rho0=1e11, c_gnd=0.0)
        model = cst.MaterialModel(mat, [[1.0, 0.0, 0.0, 0.0]])
        b, yc = mat.burgers, mat.y_c
        rng = np.random.default_rng(3)
        rho_n = rng.uniform(1e11, 5e13, size=(1, 12))
        pd = cst.PointData(model, np.zeros(1, dtype=np.int64), np.eye(3)[None], rho_n, np.zeros((1, 12)))
        inv_ell = 1.0 / pd.ell                                   # (1, 12), frozen
        for gam in (1e-6, 1e-3, 0.1 * b / yc, 20.0 * b / yc):
            rho = rho_n.copy()
            steps = 20000
            dgam = gam / steps
            f = lambda r: (inv_ell - 2.0 * yc * r) / b
            for _ in range(steps):
                k1 = f(rho)
                k2 = f(rho + 0.5 * dgam * k1)
                k3 = f(rho + 0.5 * dgam * k2)
                k4 = f(rho + dgam * k3)
                rho = rho + dgam * (k1 + 2 * k2 + 2 * k3 + k4) / 6.0
            out = cst._rho_ssd(pd, np.full((1, 12), gam))
            assert np.allclose(out, rho, rtol=1e-10, atol=0), (name, gam)
            assert np.all(out > 0)
            euler = rho_n + pd.h_ssd * gam
            if 2.0 * yc * gam / b < 1e-2:
                assert np.allclose(out, euler, rtol=1e-2 * 2.0 * yc * gam / b + 1e-14)
        # far past saturation the forward-Euler step turns negative; the exact step stays between
        # the start and the saturation density 1 / (2 y_c l)
        gam = 40.0 * b / (2.0 * yc)
        rho_hi = np.full((1, 12), 1e15)
        pd = cst.PointData(model, np.zeros(1, dtype=np.int64), np.eye(3)[None], rho_hi, np.zeros((1, 12)))
        sat = 1.0 / (2.0 * yc * pd.ell)
        out = cst._rho_ssd(pd, np.full((1, 12), gam))
        assert np.all(rho_hi + pd.h_ssd * gam < 0)
        lo, hi = np.minimum(rho_hi, sat), np.maximum(rho_hi, sat)
        assert np.all((out >= lo * (1 - 1e-12)) & (out <= hi * (1 + 1e-12)))
        assert np.allclose(out, sat, rtol=1e-12)                # exp(-40): saturated


def test_density_fixed_point_doubles_with_an_equal_gnd_forest():
    """With c_GND = 1 and a GND density equal to the SSD density on every system, the forest
    of eq. 9 is 2 x 11 rho and the fixed point of eq. 8 doubles: rho_sat = 22 / (4 y_c^2 K^2);
    eq. 7 then gives tau_c = mu b sqrt(1.975 x 2 rho).  With c_GND = 0 the GND density does not
    enter at all."""
    mat = synth.material("Cu", rho0=1e11, c_gnd=1.0)
    model = cst.MaterialModel(mat, [[1.0, 0.0, 0.0, 0.0]])
    rho_sat2 = 22.0 / (4.0 * mat.y_c ** 2 * mat.K_sim ** 2)
    pd = _uniform_point(model, rho_sat2, rho_sat2)
    assert np.allclose(cst._rho_ssd(pd, np.full((1, 12), 0.1)), rho_sat2, rtol=1e-12)
    mu = elasticity.slip_plane_shear_modulus(mat.C11, mat.C12, mat.C44)
    assert np.allclose(cst._tau_c(pd), mu * mat.burgers * np.sqrt(1.975 * 2 * rho_sat2), rtol=1e-13)
    mat0 = mat.replace(c_gnd=0.0)
    model0 = cst.MaterialModel(mat0, [[1.0, 0.0, 0.0, 0.0]])
    rho_sat = 11.0 / (4.0 * mat.y_c ** 2 * mat.K_sim ** 2)
    pd0 = _uniform_point(model0, rho_sat, 5 * rho_sat)
    assert np.allclose(cst._rho_ssd(pd0, np.full((1, 12), 0.1)), rho_sat, rtol=1e-12)
