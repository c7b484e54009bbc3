"""The reduction of the local Newton solve to six unknowns (Section 2.1, eqs. 2-6).

The slip Jacobian of the backward-Euler flow rule is J = I + D M with
M_ab = Chat_a : sym(u_b (x) w_b), Chat_a = C : P_a, P_a = sym(s_a (x) m_a), u_b = Ce s_b and
w_b = A^-T m_b.  The GPU kernels solve with J through the six-dimensional space of symmetric
tensors (Sherman-Morrison-Woodbury):
    J d = -R          <=>  (C^-1 + G) T = W R,  d_a = -R_a + D_a P_a : T
    J x = D H^T E     <=>  (C^-1 + G) T = E,    x_a = D_a P_a : T
with G T = sum_a D_a sym(u_a (x) w_a) (P_a : T).  This test checks that algebra with numpy
against a dense solve with J, for random elastic states, flow slopes and cubic constants; the
kernels themselves are checked against the oracle by the GPU tests.
"""
import numpy as np

from oracle import tables

VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def _sym_components(a, b):
    """(11, 22, 33, 23, 13, 12) components of sym(a (x) b)."""
    return np.array([0.5 * (a[i] * b[j] + a[j] * b[i]) for i, j in VOIGT])


def _contract(X, Y):
    """X : Y for symmetric tensors given by their six components."""
    w = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0])
    return float(np.sum(w * X * Y))


def _stiffness(C11, C12, C44):
    """Cubic stiffness as a map of symmetric-tensor components (tensor, not engineering, shears)."""
    S = np.zeros((6, 6))
    S[:3, :3] = C12
    S[[0, 1, 2], [0, 1, 2]] = C11
    S[[3, 4, 5], [3, 4, 5]] = 2.0 * C44
    return S


def _dense_and_rank6(seed):
    rng = np.random.default_rng(seed)
    s, m = tables.slip_systems()
    C11, C12, C44 = rng.uniform(100e3, 250e3), rng.uniform(50e3, 150e3), rng.uniform(40e3, 130e3)
    if C11 - C12 < 10e3:
        C11 = C12 + 50e3
    Cm = _stiffness(C11, C12, C44)
    Ce = np.eye(3) + 2e-3 * rng.standard_normal((3, 3))
    Ce = 0.5 * (Ce + Ce.T)
    Ainv = np.eye(3) + 2e-3 * rng.standard_normal((3, 3))
    D = 10.0 ** rng.uniform(-6, -1, 12)
    P = np.array([_sym_components(s[a], m[a]) for a in range(12)])
    Chat = P @ Cm.T                                  # Chat_a = C : P_a
    W = np.array([_sym_components(Ce @ s[b], Ainv.T @ m[b]) for b in range(12)])
    M = np.array([[_contract(Chat[a], W[b]) for b in range(12)] for a in range(12)])
    J = np.eye(12) + D[:, None] * M
    N = np.linalg.inv(Cm) + sum(D[a] * np.outer(W[a], P[a] * np.array([1, 1, 1, 2, 2, 2.0])) for a in range(12))
    return rng, J, N, D, P, W, Chat


def test_newton_step_through_six_unknowns_equals_the_dense_solve():
    for seed in range(6):
        rng, J, N, D, P, W, _ = _dense_and_rank6(seed)
        R = 1e-4 * rng.standard_normal(12)
        d_dense = np.linalg.solve(J, -R)
        T = np.linalg.solve(N, W.T @ R)
        d = -R + D * np.array([_contract(P[a], T) for a in range(12)])
        assert np.max(np.abs(d - d_dense)) <= 1e-9 * np.max(np.abs(d_dense))


def test_tangent_right_hand_sides_through_six_unknowns_equal_the_dense_solve():
    for seed in range(6):
        rng, J, N, D, P, _, Chat = _dense_and_rank6(100 + seed)
        a_vec, b_vec = rng.standard_normal(3), rng.standard_normal(3)
        E = _sym_components(a_vec, b_vec)
        x_dense = np.linalg.solve(J, D * np.array([_contract(Chat[a], E) for a in range(12)]))
        T = np.linalg.solve(N, E)
        x = D * np.array([_contract(P[a], T) for a in range(12)])
        assert np.max(np.abs(x - x_dense)) <= 1e-9 * np.max(np.abs(x_dense))
