"""The seeded grain generators (CPU): periodic power tessellations and lognormal equiaxed grains."""
import math

import numpy as np

import synth


def test_power_cells_with_equal_weights_are_the_periodic_voronoi_cells():
    n = (10, 7, 6)
    c = synth.grain_centers(synth.SplitMix64(3), 9, n)
    assert np.array_equal(synth.power_cells(n, c, np.zeros(9)), synth.periodic_voronoi(n, c))
    assert np.array_equal(synth.power_cells(n, c, np.full(9, 4.0)), synth.periodic_voronoi(n, c))


def test_lognormal_grains_meet_their_size_distribution_and_are_equiaxed():
    """40^3 voxels, 30 grains: no empty grain, every equivalent diameter within 5 % of its
    lognormal target, the spread of the diameters close to the requested 20 % of the mean, and
    every grain compact (the largest principal radius of gyration at most 2.5 times the
    smallest, measured on the periodic box around the grain's centroid)."""
    n = (40, 40, 40)
    gid, centers, target = synth.lognormal_grains(11, n, 30)
    d = synth.equivalent_diameters(gid, 30)
    assert d.min() > 0
    assert np.max(np.abs(d / target - 1)) < 0.05
    assert 0.12 < d.std() / d.mean() < 0.28
    # the spheres of the targets fill the box
    assert abs(np.sum(math.pi / 6 * target ** 3) / (40 ** 3) - 1) < 1e-12
    zz, yy, xx = np.meshgrid(*(np.arange(k) + 0.5 for k in (40, 40, 40)), indexing="ij")
    for g in range(30):
        m = gid == g
        pts = np.stack([xx[m], yy[m], zz[m]], axis=1) - centers[g]
        pts -= 40 * np.round(pts / 40)               # minimum image around the centre
        ev = np.linalg.eigvalsh(np.cov(pts.T))
        assert np.sqrt(ev.max() / ev.min()) < 2.5, (g, ev)


def test_paper_geometry_workload():
    """75^3 = 3 x 5^2 voxels, 100 grains with a 20 % lognormal spread, mean equivalent diameter
    20 um (Section 2.2)."""
    rves, path = synth.workload("paper75")
    r = rves[0]
    assert r.n == (75, 75, 75) and r.n_grains == 100
    d = synth.equivalent_diameters(r.grain_of_voxel, 100)
    assert d.min() > 0
    assert abs(d.mean() * r.voxel_size / 20e-6 - 1) < 1e-12
    assert 0.15 < d.std() / d.mean() < 0.25
    assert path.n_inc == 50 and abs(path.F_bar[-1][0] - 1.05) < 1e-12
