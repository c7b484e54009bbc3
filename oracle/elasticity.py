"""Cubic anisotropic elasticity, rotations and derived moduli (oracle; test infrastructure only).

* Hooke's law S = C : Ee (eq. 4) with the cubic stiffness of the single crystal
  (C11, C12, C44 of Table 2), rotated to the sample frame by the grain orientation.
* The grain orientation R maps crystal to sample axes: a crystal vector v_c appears in
  the sample frame as R v_c, so slip directions and normals are s = R s0, m = R m0.
* mu "parallel to the slip plane" (Table 2): the shear modulus for shear on a {111}
  plane along a <110> direction of a cubic crystal, 3 C44 (C11 - C12) / (C11 - C12 + 4 C44).
"""
from __future__ import annotations

import numpy as np


def quat_to_matrix(q) -> np.ndarray:
    """Rotation matrix of the unit quaternion (w, x, y, z) (normalised here); (..., 4) -> (..., 3, 3)."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def cubic_stiffness(C11: float, C12: float, C44: float) -> np.ndarray:
    """Fourth-order cubic stiffness C_ijkl in the crystal frame, (3, 3, 3, 3)."""
    d = np.eye(3)
    C = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    C[i, j, k, l] = (C12 * d[i, j] * d[k, l]
                                     + C44 * (d[i, k] * d[j, l] + d[i, l] * d[j, k]))
                    if i == j == k == l:
                        C[i, j, k, l] = C11
    return C


def rotate4(C: np.ndarray, R: np.ndarray) -> np.ndarray:
    """C'_ijkl = R_ip R_jq R_kr R_ls C_pqrs; R may carry leading batch axes."""
    return np.einsum("...ip,...jq,...kr,...ls,pqrs->...ijkl", R, R, R, R, C)


def slip_plane_shear_modulus(C11: float, C12: float, C44: float) -> float:
    """mu of Table 2: 3 C44 (C11 - C12) / (C11 - C12 + 4 C44)."""
    return 3.0 * C44 * (C11 - C12) / (C11 - C12 + 4.0 * C44)
