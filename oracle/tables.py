"""FCC crystallography tables of the method (oracle; test infrastructure only).

* 12 slip systems {111}<110> (Section 2.1, after eq. 7; Section 2.1 GND paragraph).
* Latent-hardening interaction matrix q^{ab} from the six coefficients of Table 1.
  The class of each pair follows the usual dislocation-junction rules: self, coplanar
  (same plane), collinear (parallel Burgers vectors on different planes), Hirth lock
  (orthogonal Burgers vectors), glissile junction (the junction Burgers vector lies in
  one of the two planes) and Lomer lock (it lies in neither).
* Dislocation-segment matrix A (eq. 11): 12 edge segments (line <112> = m x b,
  Burgers vector <110>) and 6 screw segments (line = Burgers vector = <110>),
  columns vec(b (x) t) with unit vectors, row-major vec.
* Minimum-norm inverse (eq. 13): the printed (A^T A)^{-1} A^T cannot be formed because
  A^T A (18 x 18) has rank 9; the minimiser of rho.rho subject to A rho = G is
  A^T (A A^T)^{-1} G, which is what the Lagrange-multiplier statement of eq. 13 gives.
"""
from __future__ import annotations

import numpy as np

# Slip plane normals and directions in the crystal frame (unnormalised integers).
_PLANES = [(1, 1, 1), (-1, 1, 1), (1, -1, 1), (1, 1, -1)]
_DIRS = [
    [(0, 1, -1), (-1, 0, 1), (1, -1, 0)],
    [(0, 1, -1), (1, 0, 1), (1, 1, 0)],
    [(0, 1, 1), (1, 0, -1), (1, 1, 0)],
    [(0, 1, 1), (1, 0, 1), (1, -1, 0)],
]

CLASS_NAMES = ("self", "coplanar", "collinear", "hirth", "glissile", "lomer")


def slip_systems_int():
    """Integer (n, s) pairs for the 12 systems, plane-major order."""
    n = np.array([p for p in _PLANES for _ in range(3)], dtype=np.int64)
    s = np.array([d for ds in _DIRS for d in ds], dtype=np.int64)
    return n, s


def slip_systems():
    """Unit slip directions s0 (12, 3) and unit plane normals m0 (12, 3), crystal frame."""
    n, s = slip_systems_int()
    m0 = n / np.linalg.norm(n, axis=1, keepdims=True)
    s0 = s / np.linalg.norm(s, axis=1, keepdims=True)
    return s0, m0


def schmid_tensors():
    """P0^a = s^a (x) m^a in the crystal frame, shape (12, 3, 3)."""
    s0, m0 = slip_systems()
    return np.einsum("ai,aj->aij", s0, m0)


def interaction_classes() -> np.ndarray:
    """(12, 12) class code per pair: index into CLASS_NAMES."""
    n, s = slip_systems_int()
    cls = np.zeros((12, 12), dtype=np.int64)
    for a in range(12):
        for b in range(12):
            if a == b:
                cls[a, b] = 0
                continue
            same_plane = np.array_equal(n[a], n[b])
            cross = np.cross(s[a], s[b])
            parallel = not np.any(cross)
            if same_plane:
                cls[a, b] = 1
            elif parallel:
                cls[a, b] = 2
            elif int(np.dot(s[a], s[b])) == 0:
                cls[a, b] = 3
            else:
                # 60-degree pair: the junction Burgers vector is the <110>-type one of b_a +/- b_b
                cand = [s[a] + s[b], s[a] - s[b]]
                b3 = [c for c in cand if int(np.dot(c, c)) == 2][0]
                in_plane = int(np.dot(b3, n[a])) == 0 or int(np.dot(b3, n[b])) == 0
                cls[a, b] = 4 if in_plane else 5
    return cls


def q_matrix(coeffs) -> np.ndarray:
    """q^{ab} (12 x 12) from (self, coplanar, collinear, Hirth, glissile, Lomer), Table 1."""
    c = np.asarray(coeffs, dtype=np.float64)
    return c[interaction_classes()]


def screw_directions():
    """The 6 distinct <110> directions (unit), and for each system the index of its screw."""
    _, s = slip_systems_int()
    dirs = []
    idx = np.zeros(12, dtype=np.int64)
    for a in range(12):
        found = -1
        for k, d in enumerate(dirs):
            if not np.any(np.cross(d, s[a])):
                found = k
        if found < 0:
            dirs.append(s[a].copy())
            found = len(dirs) - 1
        idx[a] = found
    d = np.array(dirs, dtype=np.float64)
    return d / np.linalg.norm(d, axis=1, keepdims=True), idx


def segment_matrix():
    """A (9 x 18): columns 0..11 edge vec(b (x) t), t = m x b; columns 12..17 screw vec(b (x) b)."""
    s0, m0 = slip_systems()
    screws, _ = screw_directions()
    cols = []
    for a in range(12):
        t = np.cross(m0[a], s0[a])
        cols.append(np.outer(s0[a], t).reshape(9))
    for d in screws:
        cols.append(np.outer(d, d).reshape(9))
    return np.array(cols).T


def min_norm_inverse(A: np.ndarray) -> np.ndarray:
    """A^+ = A^T (A A^T)^{-1} (18 x 9), the minimum-norm right inverse of eq. 13."""
    return A.T @ np.linalg.inv(A @ A.T)
