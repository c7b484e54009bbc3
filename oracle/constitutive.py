"""Finite-strain strain-gradient crystal-plasticity material point (oracle; test infrastructure only).

Section 2.1, written in the sample frame exactly as stated there:

  F = Fe Fp                                            (eq. 1)
  Lp = dFp/dt Fp^{-1} = sum_a gdot^a s^a (x) m^a       (eq. 2)
  Ee = (Fe^T Fe - I) / 2                               (eq. 3)
  S  = C : Ee                                          (eq. 4)
  tau^a = S : (s^a (x) m^a)                            (eq. 5)
  gdot^a = gdot0 (|tau^a| / tau_c^a)^(1/m) sgn(tau^a)  (eq. 6; the printed exponent "m"
           with m = 0.05 is read as the rate sensitivity, i.e. the exponent is 1/m = 20)
  tau_c^a = mu b sqrt(sum_b q^{ab} rho^b)              (eq. 7)
  rho^a = rho_SSD^a + c_gnd rho_GND^a                  (text after eq. 7; c_gnd = 1 is the
           paper's model, c_gnd = 0 its "infinite grain size" runs of Section 3)
  drho_SSD^a/dt = (1/b)(1/l^a - 2 y_c rho_SSD^a)|gdot^a|   (eq. 8)
  l^a = K / sqrt(sum_{b != a} (rho_SSD^b + c_gnd rho_GND^b))  (eq. 9, both kinds in the forest)
  P = Fe S Fe^T F^{-T}                                 (eq. 14)

Time integration over one increment dt (the paper does not state it): backward Euler in
the slip increments dg^a = gdot^a dt, the twelve unknowns of a local Newton solve,

  Fp = (I + sum_a dg^a s^a (x) m^a) Fp_n
  R^a(dg) = dg^a - dt gdot0 (|tau^a(dg)| / tau_c,n^a)^(1/m) sgn(tau^a(dg)) = 0,

with the critical stresses tau_c,n^a of eq. 7 taken from the start-of-increment
densities.  After the solve the SSD densities advance by eq. 8 integrated over the slip
|dg^a| with l^a (eq. 9) held at its start-of-increment value: eq. 8 is then linear in
rho_SSD^a, with the exact solution

  rho_SSD^a = rho_SSD,n^a exp(-x^a) + |dg^a| phi(x^a) / (b l^a),
  x^a = 2 y_c |dg^a| / b,   phi(x) = (1 - exp(-x)) / x   (phi(0) = 1),

i.e. the forward-Euler step rho_SSD,n + (1/b)(1/l - 2 y_c rho_SSD,n)|dg| times phi(x).  To first
order in |dg| the two agree; the exact form stays between rho_SSD,n and the saturation density
1/(2 y_c l) for any slip, where the forward-Euler step overshoots once x > 1 and turns negative
beyond (with y_c / b near 200 for aluminium, x exceeds 1 at |dg| = 2.6e-3).  Holding tau_c fixed inside the
increment keeps the local problem the minimiser of a strictly convex function (its
Jacobian is I + D M with D >= 0 diagonal and M the Schmid-stiffness Gram matrix), so
its root is unique; letting tau_c follow |dg| inside the solve would add the latent
interaction matrix q to the Jacobian, and q is indefinite (collinear 0.657 exceeds self
0.122), which makes that local problem lose uniqueness under multi-slip.

The GND densities enter with their start-of-increment value (they are computed from
the Nye tensor after each increment converges).  With hardening switched off tau_c^a
is held at tau0 and the SSD densities are frozen.  The consistent tangent dP/dF is
obtained here by central finite differences of the converged update; it only steers
the global Newton iteration.
"""
from __future__ import annotations

import numpy as np

from . import elasticity, tables


class MaterialModel:
    """Per-grain tables of one RVE: sample-frame stiffness and Schmid tensors."""

    def __init__(self, mat, quats, grain_elastic=None):
        self.mat = mat
        R = elasticity.quat_to_matrix(np.asarray(quats, dtype=np.float64))   # (G, 3, 3)
        self.R = R
        if grain_elastic is None:
            C0 = elasticity.cubic_stiffness(mat.C11, mat.C12, mat.C44)
            self.C = elasticity.rotate4(C0, R)                                # (G, 3,3,3,3)
        else:
            # a cubic stiffness per grain (phases of different stiffness)
            ge = np.asarray(grain_elastic, dtype=np.float64).reshape(-1, 3)
            self.C = np.stack([elasticity.rotate4(elasticity.cubic_stiffness(*ge[g]), R[g:g + 1])[0]
                               for g in range(R.shape[0])])
        s0, m0 = tables.slip_systems()
        s = np.einsum("gij,aj->gai", R, s0)
        m = np.einsum("gij,aj->gai", R, m0)
        self.P0 = np.einsum("gai,gaj->gaij", s, m)                            # (G, 12, 3, 3)
        # C : P0^a  (C has both minor symmetries, so this is C : sym(P0^a))
        self.CP0 = np.einsum("gijkl,gakl->gaij", self.C, self.P0)
        self.q = tables.q_matrix(mat.q)
        mu = mat.mu if mat.mu > 0 else elasticity.slip_plane_shear_modulus(mat.C11, mat.C12, mat.C44)
        self.mu = mu
        self.n_exp = 1.0 / mat.m_rate
        if mat.rho0 > 0:
            self.rho0 = mat.rho0
        else:
            # uniform initial SSD density that gives tau_c = tau0 through eq. 7
            self.rho0 = (mat.tau0 / (mu * mat.burgers)) ** 2 / self.q.sum(axis=1)[0]
        self.tau_c_frozen = mu * mat.burgers * np.sqrt(self.q.sum(axis=1)[0] * self.rho0)


def _inv3(A):
    """Inverse of (..., 3, 3) matrices by cofactors; a singular matrix gives inf/nan
    entries (which the local line search then rejects) instead of an exception."""
    c = np.empty_like(A)
    c[..., 0, 0] = A[..., 1, 1] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 1]
    c[..., 0, 1] = A[..., 0, 2] * A[..., 2, 1] - A[..., 0, 1] * A[..., 2, 2]
    c[..., 0, 2] = A[..., 0, 1] * A[..., 1, 2] - A[..., 0, 2] * A[..., 1, 1]
    c[..., 1, 0] = A[..., 1, 2] * A[..., 2, 0] - A[..., 1, 0] * A[..., 2, 2]
    c[..., 1, 1] = A[..., 0, 0] * A[..., 2, 2] - A[..., 0, 2] * A[..., 2, 0]
    c[..., 1, 2] = A[..., 0, 2] * A[..., 1, 0] - A[..., 0, 0] * A[..., 1, 2]
    c[..., 2, 0] = A[..., 1, 0] * A[..., 2, 1] - A[..., 1, 1] * A[..., 2, 0]
    c[..., 2, 1] = A[..., 0, 1] * A[..., 2, 0] - A[..., 0, 0] * A[..., 2, 1]
    c[..., 2, 2] = A[..., 0, 0] * A[..., 1, 1] - A[..., 0, 1] * A[..., 1, 0]
    det = A[..., 0, 0] * c[..., 0, 0] + A[..., 0, 1] * c[..., 1, 0] + A[..., 0, 2] * c[..., 2, 0]
    with np.errstate(divide="ignore", invalid="ignore"):
        return c / det[..., None, None]


class PointData:
    """Per-voxel inputs of the update, gathered once (V voxels)."""

    def __init__(self, model: MaterialModel, gid, Fp_n, rho_ssd_n, rho_gnd_n):
        mat = model.mat
        self.model = model
        self.C = model.C[gid]
        self.P0 = model.P0[gid]
        self.CP0 = model.CP0[gid]
        self.Fp_n = Fp_n
        self.rho_ssd_n = rho_ssd_n
        self.rho_gnd_n = rho_gnd_n
        forest = rho_ssd_n + mat.c_gnd * rho_gnd_n                    # (V, 12)
        others = forest.sum(axis=1, keepdims=True) - forest          # sum over b != a
        self.ell = mat.K_sim / np.sqrt(others)                        # eq. 9
        self.h_ssd = (1.0 / mat.burgers) * (1.0 / self.ell - 2.0 * mat.y_c * rho_ssd_n)  # eq. 8

    def take(self, idx):
        out = object.__new__(PointData)
        out.model = self.model
        for name in ("C", "P0", "CP0", "Fp_n", "rho_ssd_n", "rho_gnd_n", "ell", "h_ssd"):
            setattr(out, name, getattr(self, name)[idx])
        return out


def _kinematics(pd: PointData, F, dg):
    """Fp, Fe, Ee, S, tau for slip increments dg (eqs. 1-5, eq. 2 integrated)."""
    A = np.eye(3) + np.einsum("va,vaij->vij", dg, pd.P0)
    Fp = A @ pd.Fp_n
    Fe = F @ _inv3(Fp)
    Ce = np.swapaxes(Fe, 1, 2) @ Fe
    Ee = 0.5 * (Ce - np.eye(3))
    S = np.einsum("vijkl,vkl->vij", pd.C, Ee)
    tau = np.einsum("vij,vaij->va", S, pd.P0)
    return A, Fp, Fe, Ce, S, tau


def _tau_c(pd: PointData):
    """Critical resolved shear stress of eq. 7 from the start-of-increment densities."""
    model = pd.model
    mat = model.mat
    if not mat.hardening:
        return np.full(pd.rho_ssd_n.shape, model.tau_c_frozen)
    rho = pd.rho_ssd_n + mat.c_gnd * pd.rho_gnd_n
    return model.mu * mat.burgers * np.sqrt(rho @ model.q.T)


def _phi(x):
    """(1 - exp(-x)) / x, with phi(0) = 1."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    m = x > 0
    out[m] = -np.expm1(-x[m]) / x[m]
    return out


def _rho_ssd(pd: PointData, dg):
    """SSD densities at the end of the increment: eq. 8 integrated exactly over the slip
    |dg| with the mean free path (eq. 9) frozen at the start of the increment."""
    if not pd.model.mat.hardening:
        return pd.rho_ssd_n.copy()
    mat = pd.model.mat
    u = np.abs(dg)
    x = 2.0 * mat.y_c * u / mat.burgers
    return pd.rho_ssd_n + pd.h_ssd * u * _phi(x)


def residual(pd: PointData, F, dg, dt, want_jacobian=False, n_exp=None):
    """R^a = dg^a - dt gdot0 (|tau^a|/tau_c^a)^n sgn(tau^a) (n = 1/m unless given), and
    optionally the Jacobian dR/d(dg)."""
    model = pd.model
    mat = model.mat
    n = model.n_exp if n_exp is None else n_exp
    A, Fp, Fe, Ce, S, tau = _kinematics(pd, F, dg)
    tc = _tau_c(pd)
    ratio = np.abs(tau) / tc
    with np.errstate(over="ignore"):
        g = dt * mat.gamma0_dot * ratio ** n * np.sign(tau)
    R = dg - g
    if not want_jacobian:
        return R
    # dtau_a/ddg_b = -(Ce P0_b A^{-1}) : (C : P0_a)
    Ainv = _inv3(A)
    M = np.einsum("vij,vbjk,vkl->vbil", Ce, pd.P0, Ainv)
    dtau = -np.einsum("vbij,vaij->vab", M, pd.CP0)
    with np.errstate(over="ignore"):
        dg_dtau = dt * mat.gamma0_dot * n * ratio ** (n - 1.0) / tc
    J = np.eye(12)[None] - dg_dtau[:, :, None] * dtau
    return R, J


CONTINUATION_EXPONENTS = (1.0, 2.0, 4.0, 8.0, 16.0)


def _newton(pd, F, dt, dg, n_exp, tol, floor, maxit, max_step):
    """Plain Newton iterations on R = 0 at flow exponent n_exp for the voxels of pd.

    The step is shortened to max_step (max norm), then halved until |R| does not grow (at
    most 30 times).  Returns (dg, iterations, converged);
    a voxel is converged once its full step is below tol * max(|dg|, floor).  A voxel whose
    step is not finite stops and is reported as not converged.
    """
    V = F.shape[0]
    dg = dg.copy()
    iters = np.zeros(V, dtype=np.int64)
    converged = np.zeros(V, dtype=bool)
    failed = np.zeros(V, dtype=bool)
    active = np.arange(V)
    for _ in range(maxit):
        if active.size == 0:
            break
        sub = pd.take(active)
        x = dg[active]
        R, J = residual(sub, F[active], x, dt, want_jacobian=True, n_exp=n_exp)
        ok = np.all(np.isfinite(J), axis=(1, 2)) & np.all(np.isfinite(R), axis=1)
        delta = np.zeros_like(x)
        if np.any(ok):
            try:
                delta[ok] = np.linalg.solve(J[ok], -R[ok][..., None])[..., 0]
            except np.linalg.LinAlgError:
                for v in np.nonzero(ok)[0]:
                    try:
                        delta[v] = np.linalg.solve(J[v], -R[v])
                    except np.linalg.LinAlgError:
                        ok[v] = False
        ok &= np.all(np.isfinite(delta), axis=1)
        iters[active] += 1
        big = np.max(np.abs(delta), axis=1)
        delta *= np.minimum(1.0, max_step / np.maximum(big, 1e-300))[:, None]
        small = ok & (np.max(np.abs(delta), axis=1) <= tol * np.maximum(np.max(np.abs(x), axis=1), floor))
        # backtracking on |R| (skipped once the step is small: the residual is then at its
        # rounding floor and cannot be compared reliably)
        lam = np.ones(x.shape[0])
        r0 = np.linalg.norm(np.where(np.isfinite(R), R, np.inf), axis=1)
        need = ok & ~small
        trial = x + delta
        for _ls in range(30):
            idx = np.nonzero(need)[0]
            if idx.size == 0:
                break
            rt = np.linalg.norm(residual(sub.take(idx), F[active[idx]], trial[idx], dt, n_exp=n_exp), axis=1)
            good = np.isfinite(rt) & (rt <= r0[idx])
            need[idx[good]] = False
            bad = idx[~good]
            lam[bad] *= 0.5
            trial[bad] = x[bad] + lam[bad, None] * delta[bad]
        dg[active[ok]] = trial[ok]
        converged[active[small]] = True
        failed[active[~ok]] = True
        active = active[ok & ~small]
    return dg, iters, converged


def solve_slip(pd: PointData, F, dt, dg0, tol=1e-10, floor=1e-10, fast_iters=8, maxit=60,
               max_step=0.02):
    """Local Newton on the slip increments; returns (dg, iterations, converged mask).

    1. Plain Newton at the flow exponent n = 1/m from the warm start dg0, at most
       fast_iters iterations.
    2. Voxels not converged by then restart from dg0 with continuation in the exponent:
       roots at n = 1, 2, 4, 8, 16 (each to 1e-4 relative, started from the previous one),
       then Newton at n = 1/m to full tolerance.  Far from the solution the plain Jacobian
       row of an overloaded system scales with (|tau|/tau_c)^(n-1), which with n = 20 can
       exceed 1e20 and leaves J numerically singular when several systems are overloaded;
       each continuation stage starts near its root, where the rows stay moderate.
    Steps are shortened to max_step in the max norm and backtracked on |R|.  A voxel is converged once its full
    Newton step is below tol * max(|dg|, floor); that step is still applied, so the remaining
    error is of second order in it (the residual cannot be driven below its rounding floor,
    about 1e-12 of the slip increment, because the 20th power amplifies the rounding of tau).
    """
    n_final = pd.model.n_exp
    dg0 = np.asarray(dg0, dtype=np.float64)
    dg, iters, conv = _newton(pd, F, dt, dg0, n_final, tol, floor, fast_iters, max_step)
    slow = np.nonzero(~conv)[0]
    if slow.size:
        sub = pd.take(slow)
        Fs = F[slow]
        x = dg0[slow].copy()
        it_total = iters[slow].copy()
        for n_exp in CONTINUATION_EXPONENTS:
            if n_exp >= n_final:
                break
            x, it, _ = _newton(sub, Fs, dt, x, n_exp, 1e-4, floor, maxit, max_step)
            it_total += it
        x, it, c = _newton(sub, Fs, dt, x, n_final, tol, floor, maxit, max_step)
        dg[slow] = x
        iters[slow] = it_total + it
        conv[slow] = c
    return dg, iters, conv


def stress(pd: PointData, F, dg):
    """First Piola-Kirchhoff stress P = Fe S Fe^T F^{-T} (eq. 14) and the trial state."""
    A, Fp, Fe, Ce, S, tau = _kinematics(pd, F, dg)
    P = Fe @ S @ np.swapaxes(Fe, 1, 2) @ np.swapaxes(_inv3(F), 1, 2)
    return P, Fp, _rho_ssd(pd, dg), S, tau, _tau_c(pd)


def update(model: MaterialModel, gid, F, Fp_n, rho_ssd_n, rho_gnd_n, dt, dg0, chunk=8192):
    """Constitutive update of V voxels.  F, Fp_n: (V, 3, 3); densities, dg0: (V, 12).

    Returns a dict with P (V,3,3), dg (V,12), Fp, rho_ssd, S, tau, tau_c, converged, iters.
    """
    V = F.shape[0]
    out = {k: [] for k in ("P", "dg", "Fp", "rho_ssd", "S", "tau", "tau_c", "converged", "iters")}
    for lo in range(0, V, chunk):
        sl = slice(lo, min(V, lo + chunk))
        pd = PointData(model, gid[sl], Fp_n[sl], rho_ssd_n[sl], rho_gnd_n[sl])
        dg, it, conv = solve_slip(pd, F[sl], dt, dg0[sl])
        P, Fp, rho_ssd, S, tau, tc = stress(pd, F[sl], dg)
        for k, v in (("P", P), ("dg", dg), ("Fp", Fp), ("rho_ssd", rho_ssd), ("S", S),
                     ("tau", tau), ("tau_c", tc), ("converged", conv), ("iters", it)):
            out[k].append(v)
    return {k: np.concatenate(v) for k, v in out.items()}


def tangent_fd(model: MaterialModel, gid, F, Fp_n, rho_ssd_n, rho_gnd_n, dt, dg,
               step=1e-8, chunk=4096):
    """K_ijkl = dP_ij/dF_kl (V, 3, 3, 3, 3) by central differences of the converged update,
    each perturbed solve warm-started from the converged slip increments dg."""
    V = F.shape[0]
    K = np.empty((V, 3, 3, 3, 3))
    for lo in range(0, V, chunk):
        sl = slice(lo, min(V, lo + chunk))
        v = sl.stop - sl.start
        pd = PointData(model, np.repeat(gid[sl], 2), np.repeat(Fp_n[sl], 2, axis=0),
                       np.repeat(rho_ssd_n[sl], 2, axis=0), np.repeat(rho_gnd_n[sl], 2, axis=0))
        dg2 = np.repeat(dg[sl], 2, axis=0)
        for kk in range(3):
            for ll in range(3):
                Fpm = np.repeat(F[sl], 2, axis=0)
                Fpm[0::2, kk, ll] += step
                Fpm[1::2, kk, ll] -= step
                dgp, _, _ = solve_slip(pd, Fpm, dt, dg2)
                Ppm = stress(pd, Fpm, dgp)[0]
                K[sl, :, :, kk, ll] = (Ppm[0::2] - Ppm[1::2]) / (2.0 * step)
    return K


def stress_gnd_sensitivity_fd(model: MaterialModel, gid, F, Fp_n, rho_ssd_n, rho_gnd_n, dt, dg,
                              rel_step=1e-4, chunk=4096):
    """dP_ij / d rho_GND,n,b (V, 3, 3, 12) by central differences of the converged update in the
    start-of-increment GND densities, which reach the stress only through tau_c (eq. 7).  The
    step of a voxel is rel_step times its largest density; each perturbed solve is warm-started
    from the converged slip increments dg.  The stress moves by about 1e-7 of itself over the
    default step, so the local solve's convergence bound limits the quotient to a few 1e-7;
    the truncation error is of the same order."""
    V = F.shape[0]
    out = np.empty((V, 3, 3, 12))
    for lo in range(0, V, chunk):
        sl = slice(lo, min(V, lo + chunk))
        scale = np.maximum(rho_ssd_n[sl].max(axis=1), rho_gnd_n[sl].max(axis=1))
        step = rel_step * scale
        F2 = np.repeat(F[sl], 2, axis=0)
        dg2 = np.repeat(dg[sl], 2, axis=0)
        for b in range(12):
            rg = np.repeat(rho_gnd_n[sl], 2, axis=0)
            rg[0::2, b] += step
            rg[1::2, b] -= step
            pd = PointData(model, np.repeat(gid[sl], 2), np.repeat(Fp_n[sl], 2, axis=0),
                           np.repeat(rho_ssd_n[sl], 2, axis=0), rg)
            dgp, _, _ = solve_slip(pd, F2, dt, dg2)
            Ppm = stress(pd, F2, dgp)[0]
            out[sl, :, :, b] = (Ppm[0::2] - Ppm[1::2]) / (2.0 * step[:, None, None])
    return out


def density_param_sensitivity_fd(model: MaterialModel, gid, Fp_n, rho_ssd_n, rho_gnd_n, dg,
                                 rel_step=1e-4):
    """d rho_SSD / d K (row 0) and d rho_SSD / d y_c (row 1), (V, 2, 12), of the density update
    (eqs. 8-9) at fixed slip increments dg, by central differences of the material parameters.
    K and y_c do not reach the slip solve of the same increment (tau_c uses the
    start-of-increment densities), so dg stays fixed."""
    import copy
    import dataclasses
    mat = model.mat
    out = np.empty((rho_ssd_n.shape[0], 2, 12))
    for row, name in enumerate(("K_sim", "y_c")):
        base = getattr(mat, name)
        step = rel_step * abs(base)
        rho = []
        for sign in (1.0, -1.0):
            m2 = copy.copy(model)
            m2.mat = dataclasses.replace(mat, **{name: base + sign * step})
            rho.append(_rho_ssd(PointData(m2, gid, Fp_n, rho_ssd_n, rho_gnd_n), dg))
        out[:, row, :] = (rho[0] - rho[1]) / (2.0 * step)
    return out


def stress_fp_direction_fd(model: MaterialModel, gid, F, Fp_n, rho_ssd_n, rho_gnd_n, dt, dg, D,
                           step=1e-7):
    """dP/dFp_n applied to directions D (V, 3, 3), by central differences of the converged
    update in the start-of-increment plastic deformation gradient (each perturbed solve
    warm-started from dg)."""
    V = F.shape[0]
    Fpm = np.repeat(Fp_n, 2, axis=0)
    Dm = np.repeat(D, 2, axis=0)
    Fpm[0::2] += step * Dm[0::2]
    Fpm[1::2] -= step * Dm[1::2]
    pd = PointData(model, np.repeat(gid, 2), Fpm, np.repeat(rho_ssd_n, 2, axis=0),
                   np.repeat(rho_gnd_n, 2, axis=0))
    F2 = np.repeat(F, 2, axis=0)
    dgp, _, _ = solve_slip(pd, F2, dt, np.repeat(dg, 2, axis=0))
    Ppm = stress(pd, F2, dgp)[0]
    assert Ppm.shape[0] == 2 * V
    return (Ppm[0::2] - Ppm[1::2]) / (2.0 * step)
