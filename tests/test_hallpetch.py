"""Hall-Petch post-processing (Section 3, eq. 21): the fit on exact power laws (CPU) and the
size effect of a reduced sweep through the library (GPU)."""
import math

import numpy as np
import pytest

import synth
from paper_1910_01946_amd import hallpetch


def test_fit_recovers_an_exact_power_law():
    rho_i = 1.2e12
    D = np.array([10e-6, 20e-6, 40e-6, 80e-6])
    for C, x in ((0.8, 0.7), (2.5, 0.59), (0.05, 1.0)):
        s_inf = 37e6
        s_y = s_inf * (1 + C * (D * math.sqrt(rho_i)) ** (-x))
        C2, x2 = hallpetch.fit_size_effect(D, s_y, s_inf, rho_i)
        assert abs(x2 - x) < 1e-12 and abs(C2 / C - 1) < 1e-11
    with pytest.raises(ValueError):
        hallpetch.fit_size_effect(D, np.full(4, 30e6), 37e6, rho_i)   # no strengthening


def test_flow_stress_interpolates_the_curve():
    assert hallpetch.flow_stress([0.0, 0.01, 0.02], [0.0, 10.0, 14.0], 0.015) == 12.0


def test_hall_petch_workload_shares_the_microstructure_and_scales_the_voxel_size():
    rves, path, labels = synth.hall_petch_workload(n=16, n_grains=12, n_inc=10, strain_max=0.01)
    assert len(rves) == 4 * 5 and path.n_inc == 10
    for r, (m, D) in zip(rves, labels):
        assert np.array_equal(r.grain_of_voxel, rves[0].grain_of_voxel)
        d_vox = float(np.mean(synth.equivalent_diameters(r.grain_of_voxel, 12)))
        if D is None:
            assert r.material.c_gnd == 0.0
        else:
            assert r.material.c_gnd == 1.0 and abs(r.voxel_size * d_vox / D - 1) < 1e-12


@pytest.mark.gpu
def test_reduced_sweep_shows_a_grain_size_effect():
    """16^3, 12 grains, Cu and Al, four sizes and the twins, tension to 1 % in 10 increments
    (mixed form): the flow stress rises as the grains get smaller, every size is stronger than
    the twin without GND term, and the fitted exponent of eq. 21 lies in (0, 1.5)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_01946_amd as lib
    lib.lib()
    rves, path, labels = synth.hall_petch_workload(n=16, n_grains=12, n_inc=10, strain_max=0.01,
                                                   materials=("Cu", "Al"))
    res = hallpetch.run_sweep(rves, path, labels, strains=(0.01,), log=lambda s: print(s, flush=True))
    for m in ("Cu", "Al"):
        f = res["fits"][f"{m}@0.01"]
        s = f["sigma_y"]
        assert all(a > b for a, b in zip(s, s[1:])), s          # smaller D: higher stress
        assert min(f["strengthening"]) > 0
        assert 0.0 < f["x"] < 1.5, f
