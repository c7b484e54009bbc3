"""Pins of the oracle's crystallographic tables (Section 2.1, Tables 1-2, eqs. 10-13)."""
import os

import numpy as np
import pytest

import synth
from oracle import elasticity, tables


def test_slip_systems_are_fcc_111_110():
    s0, m0 = tables.slip_systems()
    n, s = tables.slip_systems_int()
    assert np.allclose(np.abs(n), 1) and np.all(np.sum(np.abs(s), axis=1) == 2)   # {111}, <110>
    assert np.allclose(np.einsum("ai,ai->a", s0, m0), 0.0)                         # s in plane
    assert np.allclose(np.linalg.norm(s0, axis=1), 1) and np.allclose(np.linalg.norm(m0, axis=1), 1)
    # 4 planes x 3 directions, every <110> direction (up to sign) in exactly two planes
    dirs = {}
    for a in range(12):
        key = tuple(s[a] if tuple(s[a]) > tuple(-s[a]) else -s[a])
        dirs.setdefault(key, set()).add(tuple(n[a]))
    assert len(dirs) == 6 and all(len(v) == 2 for v in dirs.values())


def test_interaction_classes_counts_and_row_sum():
    """Each FCC system has 1 self, 2 coplanar, 1 collinear, 2 Hirth, 4 glissile, 2 Lomer
    partners; with Table 1's coefficients every row of q sums to 1.975."""
    cls = tables.interaction_classes()
    for a in range(12):
        counts = np.bincount(cls[a], minlength=6)
        assert list(counts) == [1, 2, 1, 2, 4, 2]
    assert np.array_equal(cls, cls.T)
    q = tables.q_matrix(synth.TABLE1_Q)
    assert np.allclose(q.sum(axis=1), 1.975)


def test_lomer_pairs_have_junction_off_both_planes():
    n, s = tables.slip_systems_int()
    cls = tables.interaction_classes()
    for a in range(12):
        for b in range(12):
            if cls[a, b] == 5:
                b3 = [c for c in (s[a] + s[b], s[a] - s[b]) if c @ c == 2][0]
                assert b3 @ n[a] != 0 and b3 @ n[b] != 0
                # Lomer junction direction lies along the intersection of the planes (<110>)
                line = np.cross(n[a], n[b])
                assert line @ line == 8 or line @ line == 2 * 4


def test_segment_matrix_min_norm_inverse():
    A = tables.segment_matrix()
    assert A.shape == (9, 18)
    assert np.allclose(np.linalg.norm(A, axis=0), 1.0)       # unit b and t
    assert np.linalg.matrix_rank(A) == 9
    assert np.isclose(np.trace(A @ A.T), 18.0)
    ev = np.sort(np.linalg.eigvalsh(A @ A.T))
    assert np.allclose(ev, [1.5, 1.5, 2, 2, 2, 2, 7 / 3, 7 / 3, 7 / 3])
    Ap = tables.min_norm_inverse(A)
    assert np.allclose(A @ Ap, np.eye(9), atol=1e-13)
    # min-norm: any other solution rho + null-space vector is longer
    G = synth.random_field(3, (9,))
    rho = Ap @ G
    U, S, Vt = np.linalg.svd(A)
    null = Vt[9:]
    for k in range(5):
        z = null.T @ synth.random_field(10 + k, (9,))
        assert np.allclose(A @ (rho + z), G)
        assert np.linalg.norm(rho + z) > np.linalg.norm(rho)


def test_edge_lines_are_112_and_screw_of_system():
    s0, m0 = tables.slip_systems()
    for a in range(12):
        t = np.cross(m0[a], s0[a]) * np.sqrt(6)
        assert np.allclose(np.sort(np.abs(np.round(t))), [1, 1, 2])
    screws, idx = tables.screw_directions()
    for a in range(12):
        assert np.allclose(np.abs(screws[idx[a]] @ s0[a]), 1.0)
    assert sorted(np.bincount(idx)) == [2] * 6


def _golden_rows(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    return [l.split() for l in open(path) if l.strip() and not l.startswith("#")]


TABLE2 = {r[0]: tuple(float(v) * 1e9 for v in r[1:]) for r in _golden_rows("table2_shear_modulus.txt")}


@pytest.mark.parametrize("name", ["Cu", "Al", "Ni", "Ag"])
def test_slip_plane_shear_modulus_reproduces_table2(name):
    """The printed Table 2 shear modulus follows from the printed C_ij (to ~1 %)."""
    C11, C12, C44, mu_printed = TABLE2[name]
    mu = elasticity.slip_plane_shear_modulus(C11, C12, C44)
    assert abs(mu / mu_printed - 1) < 0.012


def test_table1_coefficients_feed_the_interaction_matrix():
    rows = {r[0]: [float(v) for v in r[1:]] for r in _golden_rows("table1_interaction.txt")}
    assert tuple(rows["q"]) == tuple(synth.TABLE1_Q)
    assert rows["gamma0_dot"][0] == synth.TABLE1_GAMMA0_DOT and rows["m"][0] == synth.TABLE1_M
    q = tables.q_matrix(rows["q"])
    # per row: 1 self, 2 coplanar, 1 collinear, 2 Hirth, 4 glissile, 2 Lomer
    assert np.allclose(q.sum(axis=1), 0.122 + 2 * 0.122 + 0.657 + 2 * 0.084 + 4 * 0.137 + 2 * 0.118)


def test_shear_modulus_is_resolved_111_110_shear_stiffness():
    """1/mu = compliance of a {111}<110> shear: apply unit shear stress on (111)[1-10]."""
    C11, C12, C44 = synth.WORKLOAD_ELASTIC["Cu"]
    C = elasticity.cubic_stiffness(C11, C12, C44)
    n = np.array([1, 1, 1]) / np.sqrt(3)
    d = np.array([1, -1, 0]) / np.sqrt(2)
    sig = np.outer(d, n) + np.outer(n, d)                  # shear stress tau = 1
    # strain from stress via the symmetric part: solve C : eps = sig in the 6-dim sym space
    basis = []
    for i in range(3):
        for j in range(i, 3):
            B = np.zeros((3, 3)); B[i, j] = B[j, i] = 1.0
            basis.append(B)
    Cm = np.array([[np.einsum("ij,ijkl,kl->", Bi, C, Bj) for Bj in basis] for Bi in basis])
    rhs = np.array([np.einsum("ij,ij->", Bi, sig) for Bi in basis])
    eps = sum(c * B for c, B in zip(np.linalg.solve(Cm, rhs), basis))
    gamma = 2 * d @ eps @ n
    assert np.isclose(1.0 / gamma, elasticity.slip_plane_shear_modulus(C11, C12, C44), rtol=1e-12)


def test_cubic_stiffness_symmetry_and_rotation_convention():
    C11, C12, C44 = 168.4e9, 121.4e9, 75.4e9
    C = elasticity.cubic_stiffness(C11, C12, C44)
    assert np.allclose(C, C.transpose(1, 0, 2, 3)) and np.allclose(C, C.transpose(2, 3, 0, 1))
    R90 = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1.0]])
    assert np.allclose(elasticity.rotate4(C, R90), C)          # cubic symmetry
    q = synth.shoemake_quaternions(synth.SplitMix64(1), 1)[0]
    R = elasticity.quat_to_matrix(q)
    assert np.allclose(R @ R.T, np.eye(3)) and np.isclose(np.linalg.det(R), 1.0)
    Cs = elasticity.rotate4(C, R)
    a, b = synth.random_field(2, (3,)), synth.random_field(3, (3,))
    # a crystal-frame pair (a_c, b_c) appears in the sample frame as (R a_c, R b_c)
    lhs = np.einsum("ijkl,ij,kl->", Cs, np.outer(R @ a, R @ b), np.outer(R @ a, R @ b))
    rhs = np.einsum("ijkl,ij,kl->", C, np.outer(a, b), np.outer(a, b))
    assert np.isclose(lhs, rhs, rtol=1e-12)
    # quaternion convention: rotation by angle t about z
    t = 0.3
    Rz = elasticity.quat_to_matrix([np.cos(t / 2), 0, 0, np.sin(t / 2)])
    assert np.allclose(Rz, [[np.cos(t), -np.sin(t), 0], [np.sin(t), np.cos(t), 0], [0, 0, 1]])
