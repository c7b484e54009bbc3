"""Independent reference solutions that pin the oracle (test infrastructure only).

None of these goes through the FFT projection:

* material_point_path: a homogeneous RVE (one grain) has a uniform solution, so the
  whole homogenization problem reduces to one material point under the mixed boundary
  condition (Section 2.2, eq. 15): the deformation-controlled components of F are
  prescribed and the stress-controlled components of P vanish.  The unknown components
  of F are found by a Newton iteration with a finite-difference Jacobian.
* laminate_path: two grains stacked along z.  Every field then depends on z only, a
  compatible fluctuation can only change the third column of F, and equilibrium
  (div P = 0) only asks the traction P e_z to be the same in both layers, so the
  discrete solution is piecewise uniform.  The 7 unknowns (third column of F in each
  layer and the free in-plane component F_yy) solve 3 traction-continuity equations, 2
  average constraints on the deformation-controlled third-column components and 2
  stress-controlled averages.
* svk_stress: a hyperelastic St. Venant-Kirchhoff first Piola-Kirchhoff stress
  P = F (C : E), E = (F^T F - I)/2, which equals eq. 14 when Fp = I.
* dense_galerkin_elastic: the Galerkin system of small-strain linear elasticity
  assembled in real space with the rotated-scheme finite-difference stencil (each
  derivative is the forward difference averaged over the 2x2 cells of the other two
  directions), solved by dense least squares.
"""
from __future__ import annotations

import numpy as np

from . import constitutive, elasticity


def svk_stress(F, C):
    E = 0.5 * (np.swapaxes(F, -1, -2) @ F - np.eye(3))
    S = np.einsum("...ijkl,...kl->...ij", C, E)
    return F @ S


def _newton_fd(fun, x0, tol=1e-15, maxit=80, h=1e-9):
    """Newton with a central-difference Jacobian and backtracking on |r|."""
    x = np.array(x0, dtype=np.float64)
    r = fun(x)
    for _ in range(maxit):
        J = np.empty((r.size, x.size))
        for j in range(x.size):
            e = np.zeros_like(x)
            e[j] = h
            J[:, j] = (fun(x + e) - fun(x - e)) / (2 * h)
        dx = np.linalg.solve(J, -r)
        if np.max(np.abs(dx)) <= tol:
            return x + dx
        lam = 1.0
        for _ls in range(30):
            r_try = fun(x + lam * dx)
            if np.linalg.norm(r_try) <= np.linalg.norm(r):
                break
            lam *= 0.5
        x = x + lam * dx
        r = r_try
    return x


class _Point:
    """One material point with its own internal variables (oracle constitutive law)."""

    def __init__(self, model, grain):
        self.model = model
        self.gid = np.array([grain])
        self.Fp = np.eye(3)[None]
        self.rho_ssd = np.full((1, 12), model.rho0)
        self.rho_gnd = np.zeros((1, 12))
        self.dg = np.zeros((1, 12))

    def stress(self, F, dt):
        out = constitutive.update(self.model, self.gid, F.reshape(1, 3, 3), self.Fp, self.rho_ssd,
                                  self.rho_gnd, dt, self.dg)
        return out

    def commit(self, out):
        self.Fp = out["Fp"]
        self.rho_ssd = out["rho_ssd"]
        self.dg = out["dg"]


def material_point_path(mat, quat, path, n_inc=None):
    """Homogeneous single-crystal response along a mixed-control load path.

    Returns a list of (F (3,3), P (3,3), S (3,3), tau (12,)) per increment."""
    model = constitutive.MaterialModel(mat, np.asarray(quat).reshape(1, 4))
    pt = _Point(model, 0)
    free = np.nonzero(np.asarray(path.mask) == 0)[0]
    F = np.eye(3).reshape(9)
    F_prev = F.copy()
    out_list = []
    n = path.n_inc if n_inc is None else n_inc
    for k in range(1, n + 1):
        Fk = F + (F - F_prev)
        fixed = np.asarray(path.mask) == 1
        Fk[fixed] = path.F_bar[k][fixed]
        F_prev = F

        def fun(x):
            G = Fk.copy()
            G[free] = x
            P = pt.stress(G.reshape(3, 3), path.dt)["P"].reshape(9)
            return P[free] - path.P_bar[k][free]

        x = _newton_fd(fun, Fk[free])
        Fk[free] = x
        out = pt.stress(Fk.reshape(3, 3), path.dt)
        pt.commit(out)
        F = Fk
        out_list.append((Fk.reshape(3, 3), out["P"][0], out["S"][0], out["tau"][0]))
    return out_list


def laminate_path(mat, quat_a, quat_b, frac_a, path, n_inc=None, elastic_svk=False):
    """Piecewise-uniform laminate solution (layers normal to z).

    Returns a list of (F_a, F_b, P_a, P_b) per increment (each (3, 3))."""
    model = constitutive.MaterialModel(mat, np.stack([quat_a, quat_b]))
    pa, pb = _Point(model, 0), _Point(model, 1)
    fa, fb = frac_a, 1.0 - frac_a
    mask = np.asarray(path.mask).reshape(3, 3)
    assert mask[2, 2] == 0 and mask[1, 1] == 0, "laminate reference expects P_yy, P_zz control"
    Fa = np.eye(3)
    Fb = np.eye(3)
    res = []
    n = path.n_inc if n_inc is None else n_inc
    for k in range(1, n + 1):
        Fbar = path.F_bar[k].reshape(3, 3)
        Pbar = path.P_bar[k].reshape(3, 3)

        def build(x):
            A = Fbar.copy()
            A[1, 1] = x[6]
            B = A.copy()
            A[:, 2] = x[0:3]
            B[:, 2] = x[3:6]
            return A, B

        def stresses(A, B):
            if elastic_svk:
                return svk_stress(A, model.C[0]), svk_stress(B, model.C[1]), None, None
            oa = pa.stress(A, path.dt)
            ob = pb.stress(B, path.dt)
            return oa["P"][0], ob["P"][0], oa, ob

        def fun(x):
            A, B = build(x)
            PA, PB, _, _ = stresses(A, B)
            r = list(PA[:, 2] - PB[:, 2])
            for i in range(2):      # deformation-controlled averages of F_xz, F_yz
                r.append(fa * A[i, 2] + fb * B[i, 2] - Fbar[i, 2])
            Pavg = fa * PA + fb * PB
            r.append((Pavg[1, 1] - Pbar[1, 1]) * 1e-11)
            r.append((Pavg[2, 2] - Pbar[2, 2]) * 1e-11)
            r[0:3] = [v * 1e-11 for v in r[0:3]]
            return np.array(r)

        x0 = np.concatenate([Fa[:, 2], Fb[:, 2], [Fa[1, 1]]])
        if k > 1:
            x0 = 2 * x0 - np.concatenate([Fa_prev[:, 2], Fb_prev[:, 2], [Fa_prev[1, 1]]])
        Fa_prev, Fb_prev = Fa, Fb
        x = _newton_fd(fun, x0)
        A, B = build(x)
        PA, PB, oa, ob = stresses(A, B)
        if oa is not None:
            pa.commit(oa)
            pb.commit(ob)
        Fa, Fb = A, B
        res.append((A, B, PA, PB))
    return res


def rotated_gradient_matrix(shape_zyx):
    """Dense real-space rotated-scheme gradient D (9V x 3V): F_ij = d_j u_i at each voxel.

    d_j f at voxel n is the average over a, b in {0, 1} of f(n + e_j + a e_p + b e_q) -
    f(n + a e_p + b e_q), (p, q) the two other directions, indices periodic."""
    nz, ny, nx = shape_zyx
    V = nx * ny * nz

    def vid(x, y, z):
        return ((z % nz) * ny + (y % ny)) * nx + (x % nx)

    D = np.zeros((9 * V, 3 * V))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                v = vid(x, y, z)
                for j in range(3):
                    others = [d for d in range(3) if d != j]
                    for a in (0, 1):
                        for b in (0, 1):
                            off = [0, 0, 0]
                            off[others[0]] = a
                            off[others[1]] = b
                            hi = list(off)
                            hi[j] += 1
                            p_hi = vid(x + hi[0], y + hi[1], z + hi[2])
                            p_lo = vid(x + off[0], y + off[1], z + off[2])
                            for i in range(3):
                                row = v * 9 + i * 3 + j
                                D[row, p_hi * 3 + i] += 0.25
                                D[row, p_lo * 3 + i] -= 0.25
    return D


def dense_galerkin_elastic(C_vox, F_bar):
    """Small-strain linear elasticity on the voxel grid: minimise sum_v (F_bar + D u)_v :
    C_v : (F_bar + D u)_v over periodic u.  C_vox: (nz, ny, nx, 3,3,3,3).  Returns F
    (nz, ny, nx, 3, 3)."""
    shape = C_vox.shape[:3]
    V = int(np.prod(shape))
    D = rotated_gradient_matrix(shape)
    Cb = np.zeros((9 * V, 9 * V))
    Cf = C_vox.reshape(V, 9, 9)
    for v in range(V):
        Cb[9 * v:9 * v + 9, 9 * v:9 * v + 9] = Cf[v]
    f0 = np.tile(np.asarray(F_bar).reshape(9), V)
    Amat = D.T @ Cb @ D
    rhs = -D.T @ (Cb @ f0)
    u = np.linalg.lstsq(Amat, rhs, rcond=1e-13)[0]
    return (f0 + D @ u).reshape(shape + (3, 3))
