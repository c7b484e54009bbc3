"""Nye tensor and geometrically necessary dislocation densities (oracle; test infrastructure only).

* Nye tensor (eq. 12, Appendix B): the curl of Fp with the rotated-scheme derivative,
  alpha_ij = eps_jml d_m Fp_il (Burgers-vector index first, as in eq. 10).  Eq. 12 and
  eq. B.2 differ by a sign and eq. B.3 writes the indices in another order; the sign does
  not reach the hardening law (only |rho| enters) and the index order of eq. 10 is the
  one that matches A.
* GND densities (eqs. 10-13): the Nye tensor is rotated to the crystal frame,
  alpha_c = R^T alpha R, and split over the 18 FCC segments with the minimum-norm
  solution rho = A^+ vec(alpha_c) / b (A built from unit vectors, so dividing by the
  Burgers vector magnitude gives densities in 1/m^2).
* Per slip system (the hardening law is written per system, eq. 7): the edge density of
  the system plus half of the screw density with the same Burgers vector (each screw
  direction is shared by two systems, so the total line length is kept).
* Reverse of the chain Fp -> alpha -> rho_GND (adjoint form): the transpose of each linear
  step (the curl with the conjugate frequency symbol, the rotation, A^+) and the sign of
  each segment density for the absolute values (0 at a zero density).
"""
from __future__ import annotations

import numpy as np

from . import elasticity, spectral, tables


def nye_tensor(Fp: np.ndarray, h: float, scheme="rotated") -> np.ndarray:
    """alpha (nz, ny, nx, 3, 3) of the plastic deformation gradient field (eq. 12)."""
    return spectral.curl(Fp, h, scheme)


def segment_densities(alpha: np.ndarray, gid: np.ndarray, quats, burgers: float) -> np.ndarray:
    """rho over the 18 segments per voxel, (nz, ny, nx, 18) (eq. 13 read as A^+)."""
    R = elasticity.quat_to_matrix(np.asarray(quats, dtype=np.float64))[gid]   # (..., 3, 3)
    alpha_c = np.einsum("...pi,...pq,...qj->...ij", R, alpha, R)
    Aplus = tables.min_norm_inverse(tables.segment_matrix())
    return np.einsum("sk,...k->...s", Aplus, alpha_c.reshape(alpha.shape[:-2] + (9,))) / burgers


def system_densities(rho_seg: np.ndarray) -> np.ndarray:
    """rho_GND per slip system: |edge_a| + |screw_k(a)| / 2, (..., 12)."""
    _, screw_of = tables.screw_directions()
    edge = np.abs(rho_seg[..., :12])
    screw = np.abs(rho_seg[..., 12:])
    return edge + 0.5 * screw[..., screw_of]


def gnd_from_fp(Fp, h, gid, quats, burgers, scheme="rotated"):
    alpha = nye_tensor(Fp, h, scheme)
    seg = segment_densities(alpha, gid, quats, burgers)
    return alpha, seg, system_densities(seg)


def curl_adjoint(A: np.ndarray, h: float) -> np.ndarray:
    """Transpose of the linear map Fp - I -> alpha of eq. 12 on real periodic fields:
    Fbar_il = sum_jm eps_jml conj(i k_m / h) A_ij, frequency by frequency."""
    k = spectral.kvector(A.shape[:3])
    sym = np.conj(1j * k / h)
    return spectral.ifft3_real(np.einsum("jml,zyxm,zyxij->zyxil", spectral.LEVI_CIVITA, sym,
                                         spectral.fft3(A)))


def gnd_adjoint(alpha, gid, quats, burgers, rho_bar):
    """alpha_bar (nz, ny, nx, 3, 3) = (d rho_GND / d alpha)^T rho_bar at the Nye tensor alpha."""
    seg = segment_densities(alpha, gid, quats, burgers)
    _, screw_of = tables.screw_directions()
    u = np.zeros_like(seg)
    u[..., :12] = np.sign(seg[..., :12]) * rho_bar
    for a in range(12):
        u[..., 12 + screw_of[a]] += 0.5 * rho_bar[..., a]
    u[..., 12:] *= np.sign(seg[..., 12:])
    Aplus = tables.min_norm_inverse(tables.segment_matrix())
    ac_bar = (np.einsum("sk,...s->...k", Aplus, u) / burgers).reshape(alpha.shape)
    R = elasticity.quat_to_matrix(np.asarray(quats, dtype=np.float64))[gid]
    return np.einsum("...ip,...pq,...jq->...ij", R, ac_bar, R)


def gnd_fp_adjoint(Fp, h, gid, quats, burgers, rho_bar):
    """Fp_bar = (d rho_GND / d Fp)^T rho_bar through the Nye tensor of Fp."""
    alpha = nye_tensor(Fp, h)
    alpha_bar = gnd_adjoint(alpha, gid, quats, burgers, rho_bar)
    return alpha_bar, curl_adjoint(alpha_bar, h)
