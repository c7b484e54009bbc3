"""Pins of the oracle's reverse of the Nye tensor / GND chain (eqs. 10-13, eq. B.3).

The transposes are checked against a dense matrix of the forward curl built column by
column, a closed form of the conjugate rotated-scheme frequency, and central differences of
the forward chain (piecewise linear in alpha and Fp, so the differences are exact up to
rounding away from sign changes of a segment density; the step is 1e-7 of the field, so the
differences carry about 1e-9 of relative rounding error and the bar is 1e-6, well below the O(1)
error of a dropped factor, a transposed rotation or a wrong screw index)."""
import numpy as np
import pytest

import synth
from oracle import nye, spectral

BURGERS = 0.256e-9


def _curl_linear(X, h):
    # the forward curl acts on Fp - I
    return spectral.curl(X + np.eye(3), h)


def test_curl_adjoint_is_the_transpose_of_the_dense_curl_matrix():
    shape = (2, 3, 4)
    h = 0.7
    n = int(np.prod(shape)) * 9
    M = np.empty((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, c] = _curl_linear(e.reshape(shape + (3, 3)), h).reshape(-1)
    Mt = np.empty((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        Mt[:, c] = nye.curl_adjoint(e.reshape(shape + (3, 3)), h).reshape(-1)
    assert np.abs(M).max() > 0.1
    assert np.allclose(Mt, M.T, atol=1e-14)


@pytest.mark.parametrize("shape", [(4, 6, 8), (5, 3, 4)])
def test_conjugate_frequency_is_the_frequency_one_voxel_back(shape):
    """conj(k_i) = k_i exp(-i (xi_x + xi_y + xi_z)): the transposed corner difference is the
    same corner difference taken one voxel back along every axis."""
    k = spectral.kvector(shape)
    nz, ny, nx = shape
    Ex = spectral.unit_roots(nx)[None, None, :]
    Ey = spectral.unit_roots(ny)[None, :, None]
    Ez = spectral.unit_roots(nz)[:, None, None]
    shift = np.conj(Ex * Ey * Ez)[..., None]
    assert np.allclose(np.conj(k), k * shift, atol=1e-15)
    A = synth.random_field(21, shape + (3, 3))
    back = np.roll(_curl_linear(A, 1.3), (1, 1, 1), axis=(0, 1, 2))
    assert np.allclose(nye.curl_adjoint(A, 1.3), back, atol=1e-13)


def _rve(shape):
    return synth.voronoi_rve(3, shape[::-1], 4, 1e-6, synth.material("Cu"))


def test_gnd_adjoint_matches_central_differences():
    shape = (3, 4, 5)
    rve = _rve(shape)
    gid = rve.grain_of_voxel
    alpha = 1e3 * synth.random_field(8, shape + (3, 3))
    d = synth.random_field(9, shape + (3, 3))
    rho_bar = synth.random_field(10, shape + (12,))

    def rho(a):
        return nye.system_densities(nye.segment_densities(a, gid, rve.quats, BURGERS))

    eps = 1e-4
    fd = np.sum(rho_bar * (rho(alpha + eps * d) - rho(alpha - eps * d))) / (2 * eps)
    ab = nye.gnd_adjoint(alpha, gid, rve.quats, BURGERS, rho_bar)
    assert abs(np.sum(ab * d) - fd) <= 1e-6 * abs(fd)
    # per voxel and per component: the gradient of one voxel's weighted density
    v = (1, 2, 3)
    for c in range(9):
        e = np.zeros(shape + (3, 3))
        e[v][c // 3, c % 3] = 1.0
        fd1 = np.sum(rho_bar * (rho(alpha + eps * e) - rho(alpha - eps * e))) / (2 * eps)
        assert abs(ab[v][c // 3, c % 3] - fd1) <= 1e-6 * np.abs(ab[v]).max()


def test_gnd_fp_adjoint_matches_central_differences():
    shape = (4, 4, 6)
    rve = _rve(shape)
    gid = rve.grain_of_voxel
    h = 2.5e-6
    Fp = np.eye(3) + 1e-3 * synth.random_field(12, shape + (3, 3))
    d = synth.random_field(13, shape + (3, 3))
    rho_bar = synth.random_field(14, shape + (12,))

    def rho(F):
        return nye.gnd_from_fp(F, h, gid, rve.quats, BURGERS)[2]

    eps = 1e-9
    fd = np.sum(rho_bar * (rho(Fp + eps * d) - rho(Fp - eps * d))) / (2 * eps)
    _, Fp_bar = nye.gnd_fp_adjoint(Fp, h, gid, rve.quats, BURGERS, rho_bar)
    assert abs(np.sum(Fp_bar * d) - fd) <= 1e-7 * abs(fd)


def test_gnd_adjoint_of_a_zero_density_is_zero():
    """At alpha = 0 every segment density is zero and the subgradient taken is 0."""
    shape = (2, 2, 2)
    rve = _rve(shape)
    ab = nye.gnd_adjoint(np.zeros(shape + (3, 3)), rve.grain_of_voxel, rve.quats, BURGERS,
                         np.ones(shape + (12,)))
    assert not ab.any()
