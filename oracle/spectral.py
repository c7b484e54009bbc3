"""Discrete differential operators in Fourier space (oracle; test infrastructure only).

Rotated scheme (Appendix A, eq. A.4).  For a grid of n_d voxels along direction d and
integer frequency index q_d, xi_d = 2 pi q_d / n_d (radians per voxel; the printed
eq. A.2 lists xi in cycles, but eq. A.4 uses tan(xi/2) and exp(i xi)) and
E_d = exp(i xi_d).  Eq. A.4 reads

    k_i = 1/4 tan(xi_i / 2) (1 + E_1)(1 + E_2)(1 + E_3),

and since tan(xi/2)(1 + exp(i xi)) = -i (exp(i xi) - 1) this equals

    k_i = 1/4 (-i)(E_i - 1) prod_{j != i} (1 + E_j),

which has no singularity at the Nyquist frequency.  The derivative of a field with
voxel size h is  d/dx_i  <->  i k_i / h  (eq. A.3 with the 1/h the printed rule omits).
In real space i k_i is the forward difference along i averaged over the 4 cells of the
2x2 stencil in the other two directions, i.e. a derivative at the voxel corner
x + h/2 (1, 1, 1).

Projection (eqs. 16-17).  The Galerkin projection onto compatible (gradient) fields is
(G : A)_ij = sum_l A_il conj(k_l) k_j / |k|^2 for every nonzero frequency with
|k| > 0.  Frequencies with two or more Nyquist coordinates have k = 0 exactly and are
projected to zero.  At the zero frequency the mixed-control rule of Section 2.2 applies:
the average of each stress-controlled component is kept (minus its prescribed value),
the average of each deformation-controlled component is removed.

Curl (eq. 12, eq. B.3).  With the Burgers-vector index first (eq. 10),
alpha_ij = eps_jml d_m Fp_il, evaluated as alpha_hat_ij = eps_jml (i k_m / h) Fp_hat_il.
"""
from __future__ import annotations

import numpy as np


def unit_roots(n: int) -> np.ndarray:
    """E(q) = exp(2 pi i q / n), q = 0..n-1, with the values at q = 0, n/4, n/2, 3n/4 exact."""
    q = np.arange(n)
    E = np.exp(2j * np.pi * q / n)
    E[0] = 1.0
    if n % 2 == 0:
        E[n // 2] = -1.0
    if n % 4 == 0:
        E[n // 4] = 1j
        E[3 * n // 4] = -1j
    return E


def modified_frequencies(shape_zyx):
    """k_x, k_y, k_z of eq. A.4 broadcast to the (nz, ny, nx) frequency grid."""
    nz, ny, nx = shape_zyx
    Ex = unit_roots(nx)[None, None, :]
    Ey = unit_roots(ny)[None, :, None]
    Ez = unit_roots(nz)[:, None, None]
    kx = 0.25 * (-1j) * (Ex - 1.0) * (1.0 + Ey) * (1.0 + Ez)
    ky = 0.25 * (-1j) * (Ey - 1.0) * (1.0 + Ex) * (1.0 + Ez)
    kz = 0.25 * (-1j) * (Ez - 1.0) * (1.0 + Ex) * (1.0 + Ey)
    return np.broadcast_arrays(kx, ky, kz)


def standard_frequencies(shape_zyx):
    """xi_x, xi_y, xi_z in radians per voxel on the (nz, ny, nx) frequency grid, each index q
    read as the signed frequency q or q - n in [-n/2, n/2); the Nyquist frequency (q = n/2 of
    an even n) gets 0: the trigonometric interpolant's derivative there is not a real field."""
    def axis(n):
        q = np.arange(n)
        xi = 2.0 * np.pi * np.where(q <= (n - 1) // 2, q, q - n) / n
        if n % 2 == 0:
            xi[n // 2] = 0.0
        return xi.astype(np.complex128)
    nz, ny, nx = shape_zyx
    return np.broadcast_arrays(axis(nx)[None, None, :], axis(ny)[None, :, None], axis(nz)[:, None, None])


def kvector(shape_zyx, scheme="rotated") -> np.ndarray:
    """(nz, ny, nx, 3) complex frequency vector: the modified frequencies of the rotated scheme
    (eq. A.4, the paper's method) or, with scheme="standard", the plain frequencies xi (the
    comparison of Appendix B)."""
    if scheme == "standard":
        kx, ky, kz = standard_frequencies(shape_zyx)
    elif scheme == "rotated":
        kx, ky, kz = modified_frequencies(shape_zyx)
    else:
        raise ValueError(scheme)
    return np.stack([kx, ky, kz], axis=-1)


def fft3(field: np.ndarray) -> np.ndarray:
    return np.fft.fftn(field, axes=(0, 1, 2))


def ifft3_real(field_hat: np.ndarray) -> np.ndarray:
    out = np.fft.ifftn(field_hat, axes=(0, 1, 2))
    return out.real


def project_hat(A_hat: np.ndarray, k: np.ndarray, mask_F, dc_target=None) -> np.ndarray:
    """Apply the projection to a spectrum A_hat (nz, ny, nx, 3, 3).

    mask_F: (9,) 1 where the average of component ij is deformation-controlled.
    dc_target: (3, 3) prescribed average of the stress-controlled components, or None.
    """
    k2 = np.sum(np.abs(k) ** 2, axis=-1)
    out = np.zeros_like(A_hat)
    nz = k2 > 0.0
    kn = k[nz]
    # u_i = sum_l A_il conj(k_l) / |k|^2, then (G:A)_ij = u_i k_j
    u = np.einsum("vil,vl->vi", A_hat[nz], np.conj(kn)) / k2[nz][:, None]
    out[nz] = np.einsum("vi,vj->vij", u, kn)
    keep = (1 - np.asarray(mask_F).reshape(3, 3)).astype(np.float64)
    nvox = A_hat.shape[0] * A_hat.shape[1] * A_hat.shape[2]
    dc = A_hat[0, 0, 0].copy()
    if dc_target is not None:
        dc = dc - nvox * np.asarray(dc_target).reshape(3, 3)
    out[0, 0, 0] = dc * keep
    return out


def project(A: np.ndarray, mask_F, dc_target=None, scheme="rotated") -> np.ndarray:
    """Real-space projection G(A) of a real tensor field (nz, ny, nx, 3, 3), eq. 17."""
    k = kvector(A.shape[:3], scheme)
    return ifft3_real(project_hat(fft3(A), k, mask_F, dc_target))


LEVI_CIVITA = np.zeros((3, 3, 3))
LEVI_CIVITA[0, 1, 2] = LEVI_CIVITA[1, 2, 0] = LEVI_CIVITA[2, 0, 1] = 1.0
LEVI_CIVITA[0, 2, 1] = LEVI_CIVITA[2, 1, 0] = LEVI_CIVITA[1, 0, 2] = -1.0


def curl(Fp: np.ndarray, h: float, scheme="rotated") -> np.ndarray:
    """alpha_ij = eps_jml d_m Fp_il with the rotated-scheme derivative (eq. 12, eq. B.3)."""
    k = kvector(Fp.shape[:3], scheme)
    Fh = fft3(Fp - np.eye(3))
    ah = np.einsum("jml,zyxm,zyxil->zyxij", LEVI_CIVITA, 1j * k / h, Fh)
    return ifft3_real(ah)


def gradient(u: np.ndarray, h: float, scheme="rotated") -> np.ndarray:
    """Rotated-scheme discrete gradient of a periodic vector field u (nz, ny, nx, 3):
    F_ij = d_j u_i, i.e. F_hat_ij = (i k_j / h) u_hat_i."""
    k = kvector(u.shape[:3], scheme)
    uh = fft3(u)
    return ifft3_real(np.einsum("zyxi,zyxj->zyxij", uh, 1j * k / h))


def derivative(f: np.ndarray, axis: int, h: float, scheme="rotated") -> np.ndarray:
    """d f / d x_axis of a real periodic scalar field f (nz, ny, nx) with the derivative of the
    scheme (axis 0 = x): i k_axis / h in Fourier space."""
    k = kvector(f.shape, scheme)[..., axis]
    return ifft3_real(fft3(f) * (1j * k / h))
