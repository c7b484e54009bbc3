"""Pins of the oracle's Galerkin-FFT homogenization (Section 2.2, eqs. 15-18) against
solutions that do not use the FFT projection."""
import numpy as np
import pytest

import synth
from oracle import elasticity, nye, reference, solver, spectral


@pytest.mark.parametrize("load", ["uniaxial", "shear", "biaxial", "stress_shear"])
def test_homogeneous_single_grain_equals_material_point(load):
    """One grain: every voxel carries the 0-D mixed-control material-point solution (solved
    directly on the free macroscopic components), for uniaxial tension, simple shear,
    equibiaxial tension and a stress-controlled shear (a nonzero prescribed P_12): the
    zero-frequency rule of the projection (keep the stress-controlled averages minus their
    targets, drop the deformation-controlled ones) is pinned by a solve that does not use it."""
    mat = synth.material("Cu", tau0=10e6, c_gnd=1.0)
    q = synth.shoemake_quaternions(synth.SplitMix64(21), 1)[0]
    rve = synth.single_crystal_rve((2, 3, 2), q, mat)
    path = {"uniaxial": lambda: synth.uniaxial_tension(0.004, 4, 1e-3),
            "shear": lambda: synth.simple_shear(0.006, 4, 1e-3),
            "biaxial": lambda: synth.biaxial_tension(0.003, 4, 1e-3),
            "stress_shear": lambda: synth.stress_controlled_shear(12e6, 4, 1.0)}[load]()
    s = solver.RVESolver(rve)
    recs = s.run(path)
    ref = reference.material_point_path(mat, q, path)
    for rec, (F, P, S, tau) in zip(recs, ref):
        assert np.allclose(np.array(rec["P_avg"]).reshape(3, 3), P, rtol=1e-9, atol=1e-3)
        assert np.allclose(np.array(rec["F_avg"]).reshape(3, 3), F, rtol=1e-12, atol=1e-13)
    assert np.abs(s.F - s.F.mean(0)).max() < 1e-13           # uniform field
    assert np.abs(s.rho_gnd).max() < 1e-3                      # uniform Fp: no GND


@pytest.mark.parametrize("plastic", [False, True])
def test_laminate_matches_piecewise_uniform_solution(plastic):
    qa = synth.shoemake_quaternions(synth.SplitMix64(31), 2)
    if plastic:
        mat = synth.material("Cu", tau0=8e6, c_gnd=0.0)
        path = synth.uniaxial_tension(0.002, 3, 1e-3)
    else:
        mat = synth.material("Ni", tau0=1e14, c_gnd=0.0)
        path = synth.uniaxial_tension(0.003, 2, 1e-3)
    n_a, nz = 3, 8
    rve = synth.laminate_rve((2, 2, nz), n_a, qa[0], qa[1], mat)
    s = solver.RVESolver(rve)
    recs = s.run(path)
    ref = reference.laminate_path(mat, qa[0], qa[1], n_a / nz, path, elastic_svk=not plastic)
    Fa, Fb, Pa, Pb = ref[-1]
    F = s.field(s.F)
    P = s.field(s.P)
    assert np.allclose(F[:n_a], Fa, rtol=0, atol=2e-12)
    assert np.allclose(F[n_a:], Fb, rtol=0, atol=2e-12)
    scale = np.abs(Pa).max()
    assert np.allclose(P[:n_a], Pa, atol=1e-8 * scale)
    assert np.allclose(P[n_a:], Pb, atol=1e-8 * scale)


def test_linear_elastic_solve_matches_dense_galerkin_assembly():
    """4x4x4, two grains, small-strain linear elasticity: one projected CG solve from F_bar
    equals the real-space Galerkin least-squares solution."""
    shape = (4, 4, 4)
    rve = synth.voronoi_rve(41, (4, 4, 4), 2, 1e-6, synth.material("Cu"))
    R = elasticity.quat_to_matrix(rve.quats)
    C0 = elasticity.cubic_stiffness(*synth.WORKLOAD_ELASTIC["Cu"])
    C = elasticity.rotate4(C0, R)[rve.grain_of_voxel]                    # (4,4,4,3,3,3,3)
    F_bar = np.array([[1e-3, 2e-4, 0], [0, -3e-4, 1e-4], [5e-5, 0, 4e-4]])
    F_ref = reference.dense_galerkin_elastic(C, F_bar)
    V = 64
    Cf = C.reshape(V, 3, 3, 3, 3)
    mask = np.ones(9)

    def apply(x):
        y = np.einsum("vijkl,vkl->vij", Cf, x)
        return spectral.project(y.reshape(shape + (3, 3)), mask).reshape(V, 3, 3)

    b = -apply(np.broadcast_to(F_bar, (V, 3, 3)).copy())
    dF, it = solver.conjugate_gradient(apply, b, 1e-14, 2000)
    F = F_bar + dF
    assert np.allclose(F.reshape(shape + (3, 3)), F_ref, rtol=0, atol=1e-15 + 1e-11 * np.abs(F_bar).max())


def _flat_project(shape):
    V = int(np.prod(shape))

    def project(A, mask):
        return spectral.project(A.reshape(tuple(shape) + (3, 3)), mask).reshape(V, 3, 3)
    return project


def test_adjoint_operator_is_the_transpose_of_the_forward_operator():
    """<y, G(K:x)> = <G(K^T:y), x> for a random non-symmetric K and random x, y in the range of
    G (where the solves act), with either zero-frequency rule: fixes the index order of K^T
    (a plain G(K:y) fails by the asymmetry)."""
    shape = (4, 6, 5)
    V = int(np.prod(shape))
    rng = np.random.default_rng(7)
    K = rng.standard_normal((V, 3, 3, 3, 3))
    x = rng.standard_normal((V, 3, 3))
    y = rng.standard_normal((V, 3, 3))
    project = _flat_project(shape)
    for mask in (np.ones(9), np.array([1, 1, 1, 1, 0, 1, 1, 1, 0])):
        x, y = project(x, mask), project(y, mask)
        fwd = project(np.einsum("vijkl,vkl->vij", K, x), mask)
        adj = solver.adjoint_operator(project, K, mask)(y)
        lhs, rhs = np.sum(y * fwd), np.sum(adj * x)
        assert abs(lhs - rhs) <= 1e-12 * np.sqrt(np.sum(y * y) * np.sum(fwd * fwd))
        wrong = project(np.einsum("vijkl,vkl->vij", K, y), mask)
        assert abs(np.sum(wrong * x) - lhs) > 1e-3 * abs(lhs)


def test_adjoint_solve_satisfies_the_transposed_system():
    """For an elastic-like tangent made non-symmetric, the adjoint CG solution solves
    G(K^T : lam) = G(g) (dense check of the residual) and differs from the solution with K."""
    shape = (4, 4, 4)
    V = 64
    rve = synth.voronoi_rve(43, shape, 2, 1e-6, synth.material("Cu"))
    R = elasticity.quat_to_matrix(rve.quats)
    C0 = elasticity.cubic_stiffness(*synth.WORKLOAD_ELASTIC["Cu"])
    K = elasticity.rotate4(C0, R)[rve.grain_of_voxel].reshape(V, 3, 3, 3, 3).copy()
    rng = np.random.default_rng(11)
    K += 0.05 * np.abs(C0).max() * rng.standard_normal(K.shape) * (rng.random(K.shape) < 0.1)
    g = rng.standard_normal((V, 3, 3))
    mask = np.array([1, 1, 1, 1, 0, 1, 1, 1, 0])
    project = _flat_project(shape)
    lam, it = solver.adjoint_solve(project, K, g, mask, 1e-13, 3000)
    res = solver.adjoint_operator(project, K, mask)(lam) - project(g, mask)
    assert np.sqrt(np.sum(res * res)) <= 1e-10 * np.sqrt(np.sum(project(g, mask) ** 2))
    lam_k, _ = solver.conjugate_gradient(lambda y: project(np.einsum("vijkl,vkl->vij", K, y), mask),
                                         project(g, mask), 1e-13, 3000)
    assert np.sqrt(np.sum((lam_k - lam) ** 2)) > 1e-3 * np.sqrt(np.sum(lam * lam))


@pytest.fixture(scope="module")
def small_run():
    rves, path = synth.workload("cu64", n_override=6, n_inc_override=50)
    rve = rves[0]
    rve.voxel_size = 5e-7
    s = solver.RVESolver(rve)
    recs = s.run(path, n_inc=2)
    return rve, path, s, recs


def test_converged_field_is_compatible_and_in_equilibrium(small_run):
    rve, path, s, recs = small_run
    F = s.field(s.F)
    P = s.field(s.P)
    # compatibility: F - <F> is a discrete gradient, so its discrete curl vanishes
    curlF = spectral.curl(F - F.mean(axis=(0, 1, 2)) + np.eye(3), 1.0)
    assert np.abs(curlF).max() < 1e-13
    # equilibrium and mixed control
    r = spectral.project(P, path.mask, path.P_bar[2].reshape(3, 3))
    assert np.abs(r).max() < 1e-9 * np.abs(P).max()
    m = path.mask.reshape(3, 3)
    assert np.allclose(F.mean(axis=(0, 1, 2)) * m, path.F_bar[2].reshape(3, 3) * m, atol=1e-14)
    assert np.all(np.abs(P.mean(axis=(0, 1, 2)) * (1 - m)) < 1e-9 * np.abs(P).max())


def test_gnd_recomputed_from_committed_fp(small_run):
    rve, path, s, recs = small_run
    alpha, seg, rho = nye.gnd_from_fp(s.field(s.Fp), rve.voxel_size, rve.grain_of_voxel,
                                      rve.quats, rve.material.burgers)
    assert np.allclose(s.field(s.rho_gnd), rho)
    assert rho.max() > 0
    # alpha scales as 1/h for a fixed Fp
    a2 = nye.nye_tensor(s.field(s.Fp), 2 * rve.voxel_size)
    assert np.allclose(a2, alpha / 2)


def test_periodic_translation_equivariance():
    rves, path = synth.workload("cu16", n_override=4)
    rve = rves[0]
    s1 = solver.RVESolver(rve)
    r1 = s1.run(path, n_inc=2)
    shifted = synth.RVE(n=rve.n, voxel_size=rve.voxel_size,
                        grain_of_voxel=np.roll(rve.grain_of_voxel, (1, 2, 3), axis=(0, 1, 2)),
                        quats=rve.quats, material=rve.material)
    s2 = solver.RVESolver(shifted)
    r2 = s2.run(path, n_inc=2)
    scale = np.abs(r1[-1]["P_avg"]).max()
    assert np.allclose(r1[-1]["P_avg"], r2[-1]["P_avg"], rtol=0, atol=1e-10 * scale)
    assert np.allclose(np.roll(s1.field(s1.F), (1, 2, 3), axis=(0, 1, 2)), s2.field(s2.F), atol=1e-12)


def test_without_gradient_term_voxel_size_does_not_matter():
    rves, path = synth.workload("cu16", n_override=4)
    rve = rves[0]
    out = []
    for h in (1e-6, 3e-5):
        rve.voxel_size = h
        out.append(solver.RVESolver(rve).run(path, n_inc=2)[-1]["P_avg"])
    assert np.allclose(out[0], out[1], rtol=0, atol=1e-11 * np.abs(out[0]).max())


def test_gradient_term_first_increment_is_size_independent_and_smaller_grains_are_harder():
    """With the GND term (c_GND = 1) the voxel size h enters only through the Nye tensor of
    the committed Fp (eq. 12 differentiates with 1/h), and the GND densities are lagged one
    increment: increment 1 starts from rho_GND = 0 and is identical for every h.  From
    increment 2 on, a smaller h (smaller grains at the same voxel count) gives larger GND
    densities, a larger forest in eqs. 7 and 9 and a strictly higher <P>_11: the grain-size
    effect the paper studies (Section 3).  A GND term entering with the wrong sign, or h
    entering anywhere else, breaks one of the two."""
    import dataclasses
    rves, path = synth.workload("cu64", n_override=4)
    rve = rves[0]
    curves = []
    for fac in (0.25, 1.0, 4.0):
        r2 = dataclasses.replace(rve, voxel_size=rve.voxel_size * fac)
        recs = solver.RVESolver(r2, newton_tol=1e-10, cg_tol=1e-8).run(path, n_inc=3)
        curves.append([rec["P_avg"][0] for rec in recs])
    first = [c[0] for c in curves]
    assert max(first) - min(first) <= 1e-13 * abs(first[0]), first
    for k in (1, 2):
        seq = [c[k] for c in curves]
        assert seq[0] > seq[1] > seq[2], (k, seq)
        assert seq[0] / seq[2] - 1 > 1e-2, (k, seq)
