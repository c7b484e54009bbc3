"""Pins of the oracle's discrete operators (Appendix A eq. A.4, eqs. 12, 16-17, eq. B.3)."""
import numpy as np
import pytest

import synth
from oracle import reference, spectral


def roll_fd(u, j, shift_axes):
    """Rotated-scheme derivative along spatial direction j of a periodic field u (nz,ny,nx,...)
    written directly in real space: forward difference along j averaged over the 2x2 cells
    spanned by the two other directions."""
    ax = {0: 2, 1: 1, 2: 0}
    out = 0.0
    others = [d for d in range(3) if d != j]
    for a in (0, 1):
        for b in (0, 1):
            sh = {others[0]: a, others[1]: b}
            base = u
            for d, s in sh.items():
                base = np.roll(base, -s, axis=ax[d])
            out = out + (np.roll(base, -1, axis=ax[j]) - base)
    return 0.25 * out


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 4, 8), (5, 3, 4)])
def test_spectral_gradient_is_the_rotated_stencil(shape):
    u = synth.random_field(11, shape + (3,))
    h = 0.7
    G = spectral.gradient(u, h)
    for j in range(3):
        fd = roll_fd(u, j, None) / h
        assert np.allclose(G[..., :, j], fd, atol=1e-13)


def test_axial_mode_is_forward_difference():
    n = 16
    x = np.arange(n)
    f = np.zeros((1, 1, n, 3))
    f[0, 0, :, 0] = np.sin(2 * np.pi * 3 * x / n) + 0.3 * np.cos(2 * np.pi * 5 * x / n)
    G = spectral.gradient(f, 1.0)
    fd = np.roll(f[0, 0, :, 0], -1) - f[0, 0, :, 0]
    assert np.allclose(G[0, 0, :, 0, 0], fd, atol=1e-14)


def test_nyquist_modes_with_two_nyquist_coordinates_have_zero_k():
    k = spectral.kvector((4, 6, 8))
    k2 = np.sum(np.abs(k) ** 2, axis=-1)
    zero = np.argwhere(k2 == 0.0)
    expect = set()
    for qz in range(4):
        for qy in range(6):
            for qx in range(8):
                nyq = (qz == 2) + (qy == 3) + (qx == 4)
                if nyq >= 2 or (qx == qy == qz == 0):
                    expect.add((qz, qy, qx))
    assert set(map(tuple, zero)) == expect


def test_curl_of_discrete_gradient_vanishes():
    u = synth.random_field(5, (8, 6, 4, 3))
    Fp = np.eye(3) + 1e-3 * spectral.gradient(u, 1.0)
    alpha = spectral.curl(Fp, 2.5)
    assert np.abs(alpha).max() < 1e-15


def test_curl_converges_to_analytic_at_voxel_corners():
    """alpha_ij = eps_jml d_m Fp_il of a smooth periodic field: second-order convergence
    to the analytic curl evaluated at x + h/2 (1,1,1)."""
    errs = []
    L = 1.0
    for n in (8, 16, 32):
        h = L / n
        c = (np.arange(n) + 0.5) * h
        Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
        w = 2 * np.pi / L

        def fields(X, Y, Z):
            Fp = np.zeros(X.shape + (3, 3))
            dFp = np.zeros(X.shape + (3, 3, 3))   # dFp[..., i, l, m] = d_m Fp_il
            Fp[..., 0, 1] = np.sin(w * Z) * np.cos(w * X)
            dFp[..., 0, 1, 2] = w * np.cos(w * Z) * np.cos(w * X)
            dFp[..., 0, 1, 0] = -w * np.sin(w * Z) * np.sin(w * X)
            Fp[..., 2, 0] = np.cos(w * Y + 0.3)
            dFp[..., 2, 0, 1] = -w * np.sin(w * Y + 0.3)
            Fp[..., 1, 2] = np.sin(w * X) * np.sin(2 * w * Y)
            dFp[..., 1, 2, 0] = w * np.cos(w * X) * np.sin(2 * w * Y)
            dFp[..., 1, 2, 1] = 2 * w * np.sin(w * X) * np.cos(2 * w * Y)
            return Fp, dFp

        Fp, _ = fields(X, Y, Z)
        _, dFc = fields(X + h / 2, Y + h / 2, Z + h / 2)
        exact = np.einsum("jml,...ilm->...ij", spectral.LEVI_CIVITA, dFc)
        alpha = spectral.curl(Fp + np.eye(3), h)
        errs.append(np.abs(alpha - exact).max() / np.abs(exact).max())
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5


def test_projection_properties():
    shape = (4, 6, 5)
    A = synth.random_field(7, shape + (3, 3))
    B = synth.random_field(8, shape + (3, 3))
    mask = synth.UNIAXIAL_MASK
    GA = spectral.project(A, mask)
    GB = spectral.project(B, mask)
    assert np.allclose(spectral.project(GA, mask), GA, atol=1e-13)          # idempotent
    assert np.isclose(np.sum(GA * B), np.sum(A * GB), rtol=1e-12)           # self-adjoint
    # gradients of periodic fields are kept; their average is zero
    u = synth.random_field(9, shape + (3,))
    grad = spectral.gradient(u, 1.0)
    assert np.allclose(spectral.project(grad, mask), grad, atol=1e-13)
    # mixed control at the zero frequency
    m = np.asarray(mask).reshape(3, 3)
    avg = GA.mean(axis=(0, 1, 2))
    assert np.allclose(avg * m, 0.0, atol=1e-15)
    assert np.allclose(avg * (1 - m), A.mean(axis=(0, 1, 2)) * (1 - m))
    target = np.diag([0.0, 0.25, -0.5])
    GT = spectral.project(A, mask, dc_target=target)
    assert np.allclose(GT.mean(axis=(0, 1, 2)) * (1 - m), (A.mean(axis=(0, 1, 2)) - target) * (1 - m))
    # a field with discretely divergence-free rows (curl of something) projects to zero
    W = synth.random_field(10, shape + (3, 3))
    khat = spectral.kvector(shape)
    Wh = np.fft.fftn(W, axes=(0, 1, 2))
    # remove the k-component of each row: Wh_ij - (Wh_il conj k_l) k_j / |k|^2
    k2 = np.sum(np.abs(khat) ** 2, -1)
    nz = k2 > 0
    proj = np.zeros_like(Wh)
    proj[nz] = np.einsum("vil,vl,vj->vij", Wh[nz], np.conj(khat[nz]), khat[nz]) / k2[nz][:, None, None]
    div_free = np.fft.ifftn(Wh - proj, axes=(0, 1, 2)).real
    div_free -= div_free.mean(axis=(0, 1, 2))
    assert np.abs(spectral.project(div_free, np.ones(9))).max() < 1e-13


def test_projection_orthogonal_to_real_space_stencil_range():
    """G(A) = 0 exactly when A is orthogonal to all discrete gradients D u: compare with the
    real-space stencil matrix."""
    shape = (3, 4, 4)
    D = reference.rotated_gradient_matrix(shape)
    A = synth.random_field(12, shape + (3, 3))
    GA = spectral.project(A, np.ones(9)).reshape(-1)
    # G is the orthogonal projector on range(D) within zero-mean fields: compare
    Q, R = np.linalg.qr(D)
    rank = np.linalg.matrix_rank(D)
    U, S, Vt = np.linalg.svd(D, full_matrices=False)
    Ur = U[:, :rank]
    assert np.allclose(GA, Ur @ (Ur.T @ A.reshape(-1)), atol=1e-13)
