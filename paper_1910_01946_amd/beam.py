"""The elastic beam benchmark of Appendix B: post-processing of the deformation field that the
library computes for the three-phase cell of synth.beam_cell (outside the homogenization path).

Strength of materials for a beam of length L whose ends are clamped and displaced by delta
against each other: w(x) = delta (3 s^2 - 2 s^3), s = x / L, so the curvature w'' = (6 delta /
L^2)(1 - 2 s) varies linearly and the bending strain eps_xx = -(y - y_0) w'' has the gradient
eps_xx,y = -w''(x), the same across the depth.  The paper compares the strain gradient that
the FFT solution gives with standard and with rotated-scheme (discrete) frequencies: both reach
the average curvature within 3 %, but the standard frequencies oscillate near the soft
layers (Gibbs), while the discrete derivative is smooth.
"""
from __future__ import annotations

import numpy as np


def frequency_vector(n: int, axis_len_index: int, scheme: str, shape_zyx):
    """i k_axis of the derivative on the (nz, ny, nx) frequency grid (axis 0 = x)."""
    nz, ny, nx = shape_zyx
    E = [np.exp(2j * np.pi * np.arange(m) / m) for m in (nx, ny, nz)]
    Ex, Ey, Ez = E[0][None, None, :], E[1][None, :, None], E[2][:, None, None]
    if scheme == "rotated":
        k = [0.25 * (-1j) * (Ex - 1) * (1 + Ey) * (1 + Ez), 0.25 * (-1j) * (Ey - 1) * (1 + Ex) * (1 + Ez),
             0.25 * (-1j) * (Ez - 1) * (1 + Ex) * (1 + Ey)]
        return 1j * np.broadcast_to(k[axis_len_index], shape_zyx)
    m = (nx, ny, nz)[axis_len_index]
    q = np.arange(m)
    xi = 2 * np.pi * np.where(q <= (m - 1) // 2, q, q - m) / m
    if m % 2 == 0:
        xi[m // 2] = 0.0
    shp = [1, 1, 1]
    shp[2 - axis_len_index] = m
    return 1j * np.broadcast_to(xi.reshape(shp), shape_zyx)


def strain_gradient(F, shape_zyx, h: float, scheme: str) -> np.ndarray:
    """eps_xx,y (nz, ny, nx) from the deformation gradient field F (9, nvox), component-major, with
    eps_xx = F_11 - 1 and the derivative of the scheme ("rotated" or "standard")."""
    exx = np.asarray(F[0]).reshape(shape_zyx) - 1.0
    d = frequency_vector(0, 1, scheme, shape_zyx)
    return np.real(np.fft.ifftn(np.fft.fftn(exx) * d)) / h


def analyze(F, shape_zyx, geom: dict, scheme: str) -> dict:
    """The beam's curvature against beam theory on its inner part (one depth away from each
    clamp), two ways: from the bending strain, kappa = -d eps_xx / dy fitted by least squares
    across the beam's rows at each x (independent of the derivative scheme: the beam's shape),
    and from the scheme's strain gradient eps_xx,y averaged over the depth; and the spread of
    eps_xx,y across the depth (beam theory: none)."""
    g = strain_gradient(F, shape_zyx, geom["h"], scheme)
    nc, nb, nd, ns = geom["n_clamp"], geom["n_beam"], geom["n_depth"], geom["n_soft"]
    exx = np.asarray(F[0]).reshape(shape_zyx)[0] - 1.0
    beam_rows = np.arange(ns, ns + nd)
    yc = (beam_rows - beam_rows.mean()) * geom["h"]
    fit_cols = np.arange(nc + nd, nc + nb - nd)
    e = exx[np.ix_(beam_rows, fit_cols)]
    kappa_fit = -(yc[:, None] * (e - e.mean(axis=0))).sum(axis=0) / (yc ** 2).sum()
    s_fit = (fit_cols + 0.5 - nc) / nb
    if scheme == "rotated":
        rows = np.arange(ns, ns + nd - 1)        # differences between two beam rows (voxel corners)
        xoff = 0.5
    else:
        rows = np.arange(ns, ns + nd)            # derivative at the voxel centres of the beam
        xoff = 0.0
    cols = np.arange(nc + nd, nc + nb - nd)
    prof = g[0][np.ix_(rows, cols)]              # (rows, cols)
    kappa = -prof.mean(axis=0)
    s = (cols + 0.5 + xoff - nc) / nb            # position along the beam
    L, delta = geom["length"], geom["delta"]
    kappa_th = 6 * delta / L ** 2 * (1 - 2 * s)
    spread = (prof.max(axis=0) - prof.min(axis=0)) / np.abs(prof.mean(axis=0)).clip(1e-300)
    q = slice(len(cols) // 8, len(cols) // 4)    # the quarter of the beam next to the clamp, x in [L/8, L/4]
    kth_fit = 6 * delta / L ** 2 * (1 - 2 * s_fit)
    return {"scheme": scheme, "mean_abs_curvature": float(np.mean(np.abs(kappa_fit))),
            "mean_abs_curvature_theory": float(np.mean(np.abs(kth_fit))),
            "curvature_error": float(np.mean(np.abs(kappa_fit)) / np.mean(np.abs(kth_fit)) - 1),
            "gradient_curvature_error": float(np.mean(np.abs(kappa)) / np.mean(np.abs(kappa_th)) - 1),
            "depth_spread_quarter": float(np.median(spread[q])),
            "profile_quarter": prof[:, q].mean(axis=1).tolist()}
