"""Galerkin-FFT homogenization of one periodic RVE (oracle; test infrastructure only).

Section 2.2.  The unknown of increment k is the deformation gradient field F_k on the
voxel grid.  Equilibrium is the projected (Galerkin) statement G(P(F) - P_bar) = 0
(eqs. 16-17) with the projection of the rotated scheme (Appendix A).  Mixed control
(eq. 15): each of the 9 macroscopic components is either a prescribed average of F
(mask 1) or a prescribed average of P (mask 0); the projection keeps the average of the
stress-controlled components (minus their target) and removes the average of the
deformation-controlled ones, so the converged field meets both kinds of constraint.

Increment k (the paper's algorithm, with our initial guess, step control and stopping rule):
  F^0 = F_{k-1} + (F_{k-1} - F_{k-2}) with the average of the deformation-controlled
        components of the added increment set to F_bar_k - F_bar_{k-1} (on the first
        increment, the uniform F_bar_1 - F_bar_0);
  P = update(F^0);  b = -G(P - P_bar_k);
  repeat: K = dP/dF at F;  solve G(K : dF) = b by conjugate gradients from dF = 0 (eq. 18);
          F_try = F + lam dF with lam = 1, 1/2, 1/4, ... until |G(P(F_try) - P_bar_k)| does not
          exceed the current residual (the first plastic increments are far outside the
          region where the full Newton step of the 20th-power flow rule converges);
          F = F_try;  stop once the applied correction has rms <= newton_tol.
Commit the internal variables of the last update (Fp, rho_SSD), then compute the Nye
tensor of Fp and the GND densities for the next increment.

Conjugate gradients (a textbook Hestenes-Stiefel loop) stop when |r| <= cg_tol |b|.
Because b and every K : p are projected, all iterates stay in the range of the
projection, where the operator is symmetric whenever K is.
"""
from __future__ import annotations

import time

import numpy as np

from . import constitutive, nye, spectral


def _dot(a, b):
    return float(np.sum(a * b))


def conjugate_gradient(apply, b, tol, maxit):
    x = np.zeros_like(b)
    r = b.copy()
    rr = _dot(r, r)
    rr0 = rr
    if rr0 == 0.0:
        return x, 0
    p = r.copy()
    it = 0
    for it in range(1, maxit + 1):
        q = apply(p)
        alpha = rr / _dot(p, q)
        x += alpha * p
        r -= alpha * q
        rr_new = _dot(r, r)
        if np.sqrt(rr_new) <= tol * np.sqrt(rr0):
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, it


def adjoint_operator(project, K, mask):
    """y -> G(K^T : y), (K^T)_(ij)(kl) = K_(kl)(ij): the transpose of the operator x -> G(K : x)
    of eq. 18 under the voxel-sum inner product (G is an orthogonal projection, so it is its
    own transpose).  project(A, mask) applies G to a (V, 3, 3) field; K is (V, 3, 3, 3, 3)."""
    def apply(y):
        return project(np.einsum("vklij,vkl->vij", K, y), mask)
    return apply


def adjoint_solve(project, K, g, mask, tol, maxit):
    """Multiplier of the linearised equilibrium for a loss with dL/dF = g: G(K^T : lam) =
    G(g), by the same conjugate gradients as the forward solve of eq. 18."""
    return conjugate_gradient(adjoint_operator(project, K, mask), project(g, mask), tol, maxit)


class RVESolver:
    """State and increment loop of one RVE (synth.RVE)."""

    def __init__(self, rve, newton_tol=1e-11, cg_tol=1e-10, max_newton=40, max_cg=5000,
                 max_backtrack=12, scheme="rotated"):
        self.rve = rve
        self.mat = rve.material
        self.model = constitutive.MaterialModel(rve.material, rve.quats, getattr(rve, "grain_elastic", None))
        self.scheme = scheme
        self.shape = rve.grain_of_voxel.shape          # (nz, ny, nx)
        self.V = int(np.prod(self.shape))
        self.gid = rve.grain_of_voxel.reshape(-1)
        self.h = rve.voxel_size
        self.newton_tol = newton_tol
        self.cg_tol = cg_tol
        self.max_newton = max_newton
        self.max_cg = max_cg
        self.max_backtrack = max_backtrack
        V = self.V
        self.F = np.tile(np.eye(3), (V, 1, 1))
        self.Fp = np.tile(np.eye(3), (V, 1, 1))
        self.rho_ssd = np.full((V, 12), self.model.rho0)
        self.rho_gnd = np.zeros((V, 12))
        self.dg = np.zeros((V, 12))
        self.P = np.zeros((V, 3, 3))
        self.alpha = np.zeros((V, 3, 3))
        self.F_bar_prev = np.eye(3).reshape(9)
        self.F_prev = None

    # ---- helpers -------------------------------------------------------------------
    def field(self, a):
        return a.reshape(self.shape + a.shape[1:])

    def flat(self, a):
        return a.reshape((self.V,) + a.shape[3:])

    def project(self, A, mask, dc_target=None):
        return self.flat(spectral.project(self.field(A), mask, dc_target, self.scheme))

    # ---- one increment -------------------------------------------------------------
    def step(self, F_bar, mask, P_bar, dt):
        F_bar = np.asarray(F_bar, dtype=np.float64).reshape(9)
        mask = np.asarray(mask).reshape(9)
        P_bar = np.asarray(P_bar, dtype=np.float64).reshape(3, 3)
        dF_macro = ((F_bar - self.F_bar_prev) * mask).reshape(3, 3)
        F = self.F + self.predictor_increment(dF_macro, mask)
        dg = self.dg.copy()
        stats = {"newton": 0, "cg": 0, "residuals": 0, "converged": False}
        t0 = time.perf_counter()
        out = self._update(F, dt, dg)
        if out is None:
            stats["error"] = "local Newton did not converge"
            return self._finish(stats, t0)
        b = -self.project(out["P"], mask, P_bar)
        stats["residuals"] += 1
        res = float(np.sqrt(np.mean(b * b)))
        for it in range(1, self.max_newton + 1):
            K = constitutive.tangent_fd(self.model, self.gid, F, self.Fp, self.rho_ssd,
                                        self.rho_gnd, dt, out["dg"])

            def apply(x):
                return self.project(np.einsum("vijkl,vkl->vij", K, x), mask)

            dF, ncg = conjugate_gradient(apply, b, self.cg_tol, self.max_cg)
            stats["newton"] += 1
            stats["cg"] += ncg
            # backtracking on the equilibrium residual: lam = 1, 1/2, 1/4, ...
            lam = 1.0
            for _ls in range(self.max_backtrack + 1):
                F_try = F + lam * dF
                out_try = self._update(F_try, dt, out["dg"])
                if out_try is not None:
                    b_try = -self.project(out_try["P"], mask, P_bar)
                    stats["residuals"] += 1
                    res_try = float(np.sqrt(np.mean(b_try * b_try)))
                    # a full correction below the tolerance is taken without a decrease
                    # test (the residual is then at its rounding floor)
                    if res_try <= res or (lam == 1.0 and np.sqrt(np.mean(dF * dF)) <= self.newton_tol):
                        break
                lam *= 0.5
            else:
                stats["error"] = "line search failed"
                return self._finish(stats, t0)
            stats["line_search_cuts"] = stats.get("line_search_cuts", 0) + _ls
            F, out, b, res = F_try, out_try, b_try, res_try
            dF_full = float(np.sqrt(np.mean(dF * dF)))
            dF_rms = lam * dF_full
            stats["dF_norm"] = dF_rms
            stats["res_norm"] = res
            # converged when the full Newton correction, not a line-search fraction of
            # it, is below the tolerance
            if lam == 1.0 and dF_full <= self.newton_tol:
                stats["converged"] = True
                break
        self._finish(stats, t0)
        if not stats["converged"]:
            return stats
        dg = out["dg"]
        # commit
        self.F_prev = self.F
        self.F = F
        self.P = out["P"]
        self.dg = dg
        self.Fp = out["Fp"]
        self.rho_ssd = out["rho_ssd"]
        self.F_bar_prev = F_bar
        alpha, _, rho_gnd = nye.gnd_from_fp(self.field(self.Fp), self.h, self.rve.grain_of_voxel,
                                            self.rve.quats, self.mat.burgers, scheme=self.scheme)
        self.alpha = self.flat(alpha)
        self.rho_gnd = self.flat(rho_gnd)
        return stats

    def predictor_increment(self, dF_macro, mask):
        """Initial guess of the field increment: the previous increment's field increment with
        its averages over the deformation-controlled components replaced by the new target
        increment (both parts stay compatible); the uniform target increment on the first
        increment."""
        if self.F_prev is None:
            return np.broadcast_to(dF_macro, self.F.shape)
        D = self.F - self.F_prev
        m = np.asarray(mask).reshape(3, 3).astype(np.float64)
        return D + m * (dF_macro - D.mean(axis=0))

    def _update(self, F, dt, dg0):
        out = constitutive.update(self.model, self.gid, F, self.Fp, self.rho_ssd, self.rho_gnd,
                                  dt, dg0)
        self._local_iters = max(getattr(self, "_local_iters", 0), int(out["iters"].max()))
        return out if np.all(out["converged"]) else None

    def _finish(self, stats, t0):
        stats["seconds"] = time.perf_counter() - t0
        stats["voxel_iterations"] = self.V * (stats["residuals"] + stats["cg"])
        stats["local_iters_max"] = getattr(self, "_local_iters", 0)
        self._local_iters = 0
        return stats

    # ---- outputs -------------------------------------------------------------------
    def macro(self):
        """<P>, <F> and the macroscopic Cauchy stress <P><F>^T / det<F> (row-major 9-vectors)."""
        P_avg = self.P.mean(axis=0)
        F_avg = self.F.mean(axis=0)
        sigma = P_avg @ F_avg.T / np.linalg.det(F_avg)
        return P_avg.reshape(9), F_avg.reshape(9), sigma.reshape(9)

    def run(self, path, n_inc=None, log=None):
        """Run the load path; returns a list of per-increment records."""
        recs = []
        n = path.n_inc if n_inc is None else n_inc
        for k in range(1, n + 1):
            st = self.step(path.F_bar[k], path.mask, path.P_bar[k], path.dt)
            if not st["converged"]:
                raise RuntimeError(f"increment {k} did not converge: {st}")
            P_avg, F_avg, sigma = self.macro()
            rec = dict(increment=k, P_avg=P_avg.tolist(), F_avg=F_avg.tolist(),
                       sigma=sigma.tolist(), **{k2: v for k2, v in st.items()})
            recs.append(rec)
            if log:
                log(rec)
        return recs
