"""Seeded synthetic inputs shared by the oracle and the GPU library's tests and benchmark.

This module holds no arithmetic of the homogenization method itself: it only draws
random numbers and lays out microstructures, material constants and load paths.

* Random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), mapped to [0, 1)
  as (x >> 11) * 2**-53.
* Microstructure: periodic Voronoi tessellation of seeded uniform grain centers,
  distances measured from voxel centers (i + 1/2) with the minimum-image rule,
  ties resolved to the lowest grain id.  The paper generates its equiaxed RVEs
  with Dream3D (Section 2.2); those files are not available, so seeded Voronoi
  RVEs stand in for them.
* Orientations: uniform random rotations drawn as unit quaternions with
  Shoemake's method (Graphics Gems III, 1992), stored (w, x, y, z) and mapping
  the crystal frame to the sample frame.
* Materials: elastic constants of the workloads (Cu, Al, Ag, Ni), the dislocation
  parameters of Table 2 and the common parameters of Table 1.
* Load path: uniaxial tension along x at constant engineering strain rate
  (Section 3): F_11(t) = 1 + rate * t, shear components held at zero, lateral
  normal stresses P_22 = P_33 = 0.

Voxel arrays are shaped (nz, ny, nx) so that the flat C-order index has x fastest.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 generator (Steele, Lea & Flood 2014)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniforms(self, n: int) -> np.ndarray:
        return np.array([self.uniform() for _ in range(n)], dtype=np.float64)


def shoemake_quaternions(rng: SplitMix64, n: int) -> np.ndarray:
    """n uniform random unit quaternions (w, x, y, z), three draws each."""
    q = np.empty((n, 4))
    for g in range(n):
        u1, u2, u3 = rng.uniform(), rng.uniform(), rng.uniform()
        a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
        t2, t3 = 2.0 * math.pi * u2, 2.0 * math.pi * u3
        q[g] = (b * math.cos(t3), a * math.sin(t2), a * math.cos(t2), b * math.sin(t3))
    return q


def grain_centers(rng: SplitMix64, n_grains: int, n: Sequence[int]) -> np.ndarray:
    """Uniform centers in [0, n_x) x [0, n_y) x [0, n_z), voxel units, (x, y, z) per row."""
    c = np.empty((n_grains, 3))
    for g in range(n_grains):
        for d in range(3):
            c[g, d] = rng.uniform() * n[d]
    return c


def periodic_voronoi(n: Sequence[int], centers: np.ndarray) -> np.ndarray:
    """Grain id per voxel, shape (nz, ny, nx), int32.

    Distance from the voxel center (i + 1/2) to each grain center with the
    periodic minimum-image convention; np.argmin keeps the lowest id on ties.
    """
    nx, ny, nz = int(n[0]), int(n[1]), int(n[2])
    out = np.empty((nz, ny, nx), dtype=np.int32)
    xs = np.arange(nx) + 0.5
    ys = np.arange(ny) + 0.5

    def wrap(d, L):
        d = np.abs(d)
        return np.minimum(d, L - d)

    dx = wrap(xs[None, :] - centers[:, 0:1], nx) ** 2          # (G, nx)
    dy = wrap(ys[None, :] - centers[:, 1:2], ny) ** 2          # (G, ny)
    for k in range(nz):
        dz = wrap((k + 0.5) - centers[:, 2], nz) ** 2          # (G,)
        d2 = dz[:, None, None] + dy[:, :, None] + dx[:, None, :]  # (G, ny, nx)
        out[k] = np.argmin(d2, axis=0).astype(np.int32)
    return out


def power_cells(n: Sequence[int], centers: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Grain id per voxel, shape (nz, ny, nx): the periodic power (Laguerre) tessellation that
    assigns a voxel centre x to the grain minimising |x - c_g|^2 - w_g (minimum image; lowest
    id on ties).  Equal weights give the Voronoi tessellation of periodic_voronoi."""
    nx, ny, nz = int(n[0]), int(n[1]), int(n[2])
    out = np.empty((nz, ny, nx), dtype=np.int32)
    xs = np.arange(nx) + 0.5
    ys = np.arange(ny) + 0.5

    def wrap(d, L):
        d = np.abs(d)
        return np.minimum(d, L - d)

    dx = wrap(xs[None, :] - centers[:, 0:1], nx) ** 2
    dy = wrap(ys[None, :] - centers[:, 1:2], ny) ** 2
    w = np.asarray(weights, dtype=np.float64)
    for k in range(nz):
        dz = wrap((k + 0.5) - centers[:, 2], nz) ** 2 - w
        d2 = dz[:, None, None] + dy[:, :, None] + dx[:, None, :]
        out[k] = np.argmin(d2, axis=0).astype(np.int32)
    return out


def _periodic_centroids(gid: np.ndarray, n_grains: int) -> np.ndarray:
    """Centroid of every grain on the periodic box (per axis, the mean of the voxel-centre
    angles 2 pi x / L mapped back to a coordinate), (x, y, z) per row; empty grains give 0."""
    nz, ny, nx = gid.shape
    ids = gid.reshape(-1)
    out = np.zeros((n_grains, 3))
    axes = ((np.arange(nx) + 0.5)[None, None, :], (np.arange(ny) + 0.5)[None, :, None],
            (np.arange(nz) + 0.5)[:, None, None])
    for d, (c, L) in enumerate(zip(axes, (nx, ny, nz))):
        ang = np.broadcast_to(2.0 * math.pi * c / L, gid.shape).reshape(-1)
        s = np.bincount(ids, np.sin(ang), n_grains)
        co = np.bincount(ids, np.cos(ang), n_grains)
        out[:, d] = (np.arctan2(s, co) % (2.0 * math.pi)) * L / (2.0 * math.pi)
    return out


def lognormal_grains(seed: int, n: Sequence[int], n_grains: int, sd_frac: float = 0.2, sweeps: int = 20):
    """Periodic equiaxed grains whose equivalent-sphere diameters follow a lognormal
    distribution with standard deviation sd_frac times the mean (Section 2.2 describes such
    RVEs, made with Dream3D, which is not available here).

    Target diameters are drawn lognormal (Box-Muller normals from SplitMix64) and scaled so that
    their spheres fill the box; centres start uniform.  The cells form a periodic power
    (Laguerre) tessellation, relaxed over a few sweeps: every non-empty cell's centre moves to
    its centroid (which keeps the grains equiaxed) and its weight grows by (D_target^2 -
    D^2) / 4, D the current equivalent diameter (which drives the cell volumes to their
    targets; 20 sweeps bring every diameter within about 2 % of its target at 75^3 with 100
    grains).  Returns (grain id per voxel (nz, ny, nx), centres, target diameters in voxels)."""
    rng = SplitMix64(seed)
    centers = grain_centers(rng, n_grains, n)
    z = gaussian_noise(seed + 7919, n_grains)
    s2 = math.log(1.0 + sd_frac ** 2)
    d = np.exp(math.sqrt(s2) * z - 0.5 * s2)                      # mean 1, sd sd_frac
    vol = float(n[0] * n[1] * n[2])
    d *= (6.0 * vol / (math.pi * np.sum(d ** 3))) ** (1.0 / 3.0)  # spheres fill the box
    w = np.zeros(n_grains)
    gid = power_cells(n, centers, w)
    for _ in range(sweeps):
        d_now = equivalent_diameters(gid, n_grains)
        full = d_now > 0
        centers[full] = _periodic_centroids(gid, n_grains)[full]
        w += 0.25 * (d ** 2 - d_now ** 2)
        gid = power_cells(n, centers, w)
    return gid, centers, d


def equivalent_diameters(gid: np.ndarray, n_grains: int) -> np.ndarray:
    """Equivalent-sphere diameter (voxels) of every grain of a grain map."""
    counts = np.bincount(gid.reshape(-1), minlength=n_grains).astype(np.float64)
    return (6.0 * counts / math.pi) ** (1.0 / 3.0)


# --------------------------------------------------------------------------------------
# Materials.  Elastic constants in Pa, lengths in m.
# --------------------------------------------------------------------------------------
# Table 1 (common to all FCC crystals): reference slip rate, rate sensitivity and the six
# interaction coefficients (self, coplanar, collinear, Hirth, glissile, Lomer).
TABLE1_GAMMA0_DOT = 1.0e-3
TABLE1_M = 0.05
TABLE1_Q = (0.122, 0.122, 0.657, 0.084, 0.137, 0.118)

# Table 2 dislocation parameters: Burgers vector, effective annihilation distance y_c,
# similitude coefficient K.
TABLE2_DISLOCATION = {
    "Cu": (0.256e-9, 15.0e-9, 6.0),
    "Al": (0.286e-9, 56.0e-9, 9.0),
    "Ni": (0.250e-9, 14.0e-9, 11.0),
    "Ag": (0.288e-9, 12.5e-9, 5.0),
}
# Table 2 elastic constants (C11, C12, C44) and the printed slip-plane shear modulus.
TABLE2_ELASTIC = {
    "Cu": (169e9, 122e9, 75.3e9),
    "Al": (108e9, 61.3e9, 28.0e9),
    "Ni": (249e9, 155e9, 114e9),
    "Ag": (124e9, 93.7e9, 46.1e9),
}
TABLE2_MU = {"Cu": 30.5e9, "Al": 25.0e9, "Ni": 58.4e9, "Ag": 19.5e9}
# Elastic constants of the benchmark workloads (they differ slightly from Table 2).
WORKLOAD_ELASTIC = {
    "Cu": (168.4e9, 121.4e9, 75.4e9),
    "Al": (108e9, 62e9, 28.3e9),
    "Ag": (124e9, 93.4e9, 46.1e9),
    "Ni": (246.5e9, 147.3e9, 124.7e9),
}


@dataclasses.dataclass
class Material:
    C11: float
    C12: float
    C44: float
    burgers: float
    y_c: float
    K_sim: float
    gamma0_dot: float = TABLE1_GAMMA0_DOT
    m_rate: float = TABLE1_M
    q: tuple = TABLE1_Q
    tau0: float = 0.0      # Pa; > 0: sets the initial SSD density per system
    rho0: float = 0.0      # 1/m^2 per system; used when > 0 (overrides tau0)
    c_gnd: float = 1.0     # weight of the GND density in the hardening law (0: no gradient)
    hardening: int = 1     # 1: Taylor/Kocks-Mecking hardening; 0: tau_c frozen at tau0
    mu: float = 0.0        # Pa; <= 0: computed from the cubic constants

    def replace(self, **kw) -> "Material":
        return dataclasses.replace(self, **kw)


def material(name: str, elastic: str = "workload", **kw) -> Material:
    C = (WORKLOAD_ELASTIC if elastic == "workload" else TABLE2_ELASTIC)[name]
    b, yc, K = TABLE2_DISLOCATION[name]
    return Material(C11=C[0], C12=C[1], C44=C[2], burgers=b, y_c=yc, K_sim=K, **kw)


# --------------------------------------------------------------------------------------
# RVEs and load paths
# --------------------------------------------------------------------------------------
@dataclasses.dataclass
class RVE:
    n: tuple                 # (nx, ny, nz)
    voxel_size: float        # h, m
    grain_of_voxel: np.ndarray  # (nz, ny, nx) int32
    quats: np.ndarray        # (n_grains, 4) (w, x, y, z), crystal -> sample
    material: Material
    seed: int = 0
    grain_elastic: np.ndarray = None  # (n_grains, 3) C11, C12, C44 per grain (Pa); None: the material's

    @property
    def n_grains(self) -> int:
        return self.quats.shape[0]

    @property
    def n_vox(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


def voronoi_rve(seed: int, n, n_grains: int, voxel_size: float, mat: Material) -> RVE:
    """Seeded periodic Voronoi RVE: 3 draws per grain center, then 3 per orientation."""
    n = tuple(int(v) for v in (n if hasattr(n, "__len__") else (n, n, n)))
    rng = SplitMix64(seed)
    centers = grain_centers(rng, n_grains, n)
    quats = shoemake_quaternions(rng, n_grains)
    gid = periodic_voronoi(n, centers)
    return RVE(n=n, voxel_size=voxel_size, grain_of_voxel=gid, quats=quats, material=mat, seed=seed)


def single_crystal_rve(n, quat, mat: Material, voxel_size: float = 1e-6) -> RVE:
    n = tuple(int(v) for v in (n if hasattr(n, "__len__") else (n, n, n)))
    gid = np.zeros((n[2], n[1], n[0]), dtype=np.int32)
    return RVE(n=n, voxel_size=voxel_size, grain_of_voxel=gid,
               quats=np.asarray(quat, dtype=np.float64).reshape(1, 4), material=mat)


def laminate_rve(n, n_layers_a: int, quat_a, quat_b, mat: Material, voxel_size: float = 1e-6) -> RVE:
    """Two grains stacked along z: layers k < n_layers_a are grain 0, the rest grain 1."""
    n = tuple(int(v) for v in (n if hasattr(n, "__len__") else (n, n, n)))
    gid = np.ones((n[2], n[1], n[0]), dtype=np.int32)
    gid[:n_layers_a] = 0
    quats = np.stack([np.asarray(quat_a, float), np.asarray(quat_b, float)])
    return RVE(n=n, voxel_size=voxel_size, grain_of_voxel=gid, quats=quats, material=mat)


# Uniaxial tension along x: F-controlled 11,12,13,21,23,31,32; P-controlled 22, 33.
UNIAXIAL_MASK = np.array([1, 1, 1, 1, 0, 1, 1, 1, 0], dtype=np.uint8)


@dataclasses.dataclass
class LoadPath:
    F_bar: np.ndarray   # (n_inc + 1, 9) macroscopic F targets (row-major), index 0 = t0
    P_bar: np.ndarray   # (n_inc + 1, 9) macroscopic P targets where mask == 0
    mask: np.ndarray    # (9,) uint8, 1 = F-controlled
    dt: float

    @property
    def n_inc(self) -> int:
        return self.F_bar.shape[0] - 1


def uniaxial_tension(strain_max: float, n_inc: int, rate: float) -> LoadPath:
    dt = strain_max / (n_inc * rate)
    F = np.tile(np.eye(3).reshape(9), (n_inc + 1, 1))
    F[:, 0] = 1.0 + rate * dt * np.arange(n_inc + 1)
    return LoadPath(F_bar=F, P_bar=np.zeros((n_inc + 1, 9)), mask=UNIAXIAL_MASK.copy(), dt=dt)


# Simple shear in the x-y plane: F-controlled shears (F_12 = rate t, the others 0), normal
# stresses P_11 = P_22 = P_33 = 0.
SHEAR_MASK = np.array([0, 1, 1, 1, 0, 1, 1, 1, 0], dtype=np.uint8)
# Equibiaxial tension in x and y: F_11 = F_22 = 1 + rate t, shears held at 0, P_33 = 0.
BIAXIAL_MASK = np.array([1, 1, 1, 1, 1, 1, 1, 1, 0], dtype=np.uint8)
# Stress-controlled shear: P_12 prescribed (a ramp), P_11 = P_22 = P_33 = 0, the other shears of F
# held at 0 (F_12 follows from equilibrium).
STRESS_SHEAR_MASK = np.array([0, 0, 1, 1, 0, 1, 1, 1, 0], dtype=np.uint8)


def simple_shear(gamma_max: float, n_inc: int, rate: float) -> LoadPath:
    dt = gamma_max / (n_inc * rate)
    F = np.tile(np.eye(3).reshape(9), (n_inc + 1, 1))
    F[:, 1] = rate * dt * np.arange(n_inc + 1)
    return LoadPath(F_bar=F, P_bar=np.zeros((n_inc + 1, 9)), mask=SHEAR_MASK.copy(), dt=dt)


def biaxial_tension(strain_max: float, n_inc: int, rate: float) -> LoadPath:
    dt = strain_max / (n_inc * rate)
    F = np.tile(np.eye(3).reshape(9), (n_inc + 1, 1))
    F[:, 0] = F[:, 4] = 1.0 + rate * dt * np.arange(n_inc + 1)
    return LoadPath(F_bar=F, P_bar=np.zeros((n_inc + 1, 9)), mask=BIAXIAL_MASK.copy(), dt=dt)


def stress_controlled_shear(tau_max: float, n_inc: int, dt: float) -> LoadPath:
    P = np.zeros((n_inc + 1, 9))
    P[:, 1] = tau_max * np.arange(n_inc + 1) / n_inc
    return LoadPath(F_bar=np.tile(np.eye(3).reshape(9), (n_inc + 1, 1)), P_bar=P,
                    mask=STRESS_SHEAR_MASK.copy(), dt=dt)


# --------------------------------------------------------------------------------------
# The benchmark workloads
# --------------------------------------------------------------------------------------
def voxel_size_for(d: float, n_grains: int, n: int) -> float:
    """Grain size d read as L / n_grains^(1/3): voxel size h = d * n_grains^(1/3) / n."""
    return d * n_grains ** (1.0 / 3.0) / n


SWEEP_SIZES = (32, 40, 48, 64, 72, 80, 96)
SWEEP_MATERIALS = ("Cu", "Ag", "Ni")


def workload(name: str, n_override=None, n_inc_override=None):
    """Return (list of RVEs, LoadPath, description) for a named benchmark workload.

    cu16:     16^3, 8 grains, Cu, tau0 = 10 MPa, no gradient term, 1% in 20 increments at 1e-3/s.
    cu64:     64^3, 64 grains, Cu, d = 50 um, rho_i = 1.2e12 (1e11 per system), 5% in 50 at 1e-4/s.
    al128:    128^3, 200 grains, Al, d = 20 um, 5% in 50 increments at 1e-4/s.
    sweep32:  32 RVEs of uneven size (32^3..96^3), 16..128 grains, d log-uniform in
              [10, 200] um, Cu/Ag/Ni, 3% in 30 increments at 1e-4/s (a grain-size sweep).
    cu64g100: 64^3, 100 grains, Cu, d = 30 um, 4% in 40 increments at 1e-4/s.
    paper75:  75^3 (3 x 5^2), 100 equiaxed grains with lognormal equivalent diameters (sd 20 %
              of the mean), mean equivalent diameter 20 um, Cu, rho_i = 1.2e12, 5% in 50 at 1e-4/s.
    """
    if name == "cu16":
        n = n_override or 16
        mat = material("Cu", tau0=10e6, c_gnd=0.0)
        rves = [voronoi_rve(101, n, 8, voxel_size_for(50e-6, 8, n), mat)]
        path = uniaxial_tension(0.01, n_inc_override or 20, 1e-3)
    elif name == "cu64":
        n = n_override or 64
        mat = material("Cu", rho0=1e11, c_gnd=1.0)
        rves = [voronoi_rve(102, n, 64, voxel_size_for(50e-6, 64, n), mat)]
        path = uniaxial_tension(0.05, n_inc_override or 50, 1e-4)
    elif name == "al128":
        n = n_override or 128
        mat = material("Al", rho0=1e11, c_gnd=1.0)
        rves = [voronoi_rve(103, n, 200, voxel_size_for(20e-6, 200, n), mat)]
        path = uniaxial_tension(0.05, n_inc_override or 50, 1e-4)
    elif name == "sweep32":
        rves = []
        for r in range(32):
            rng = SplitMix64(1040 + r)
            nr = SWEEP_SIZES[min(int(rng.uniform() * len(SWEEP_SIZES)), len(SWEEP_SIZES) - 1)]
            ng = 16 + min(int(rng.uniform() * 113), 112)
            d = 10e-6 * math.exp(rng.uniform() * math.log(20.0))
            if n_override:
                nr = n_override
            mat = material(SWEEP_MATERIALS[r % 3], rho0=1e11, c_gnd=1.0)
            centers = grain_centers(rng, ng, (nr, nr, nr))
            quats = shoemake_quaternions(rng, ng)
            gid = periodic_voronoi((nr, nr, nr), centers)
            rves.append(RVE(n=(nr, nr, nr), voxel_size=voxel_size_for(d, ng, nr),
                            grain_of_voxel=gid, quats=quats, material=mat, seed=1040 + r))
        path = uniaxial_tension(0.03, n_inc_override or 30, 1e-4)
    elif name == "paper75":
        n = n_override or 75
        mat = material("Cu", rho0=1e11, c_gnd=1.0)
        gid, _, _ = lognormal_grains(106, (n, n, n), 100)
        quats = shoemake_quaternions(SplitMix64(1106), 100)
        d_vox = float(np.mean(equivalent_diameters(gid, 100)))
        rves = [RVE(n=(n, n, n), voxel_size=20e-6 / d_vox, grain_of_voxel=gid, quats=quats, material=mat,
                    seed=106)]
        path = uniaxial_tension(0.05, n_inc_override or 50, 1e-4)
    elif name == "cu64g100":
        n = n_override or 64
        mat = material("Cu", rho0=1e11, c_gnd=1.0)
        rves = [voronoi_rve(105, n, 100, voxel_size_for(30e-6, 100, n), mat)]
        path = uniaxial_tension(0.04, n_inc_override or 40, 1e-4)
    else:
        raise ValueError(name)
    return rves, path


HALL_PETCH_MATERIALS = ("Cu", "Al", "Ag", "Ni")
HALL_PETCH_SIZES = (10e-6, 20e-6, 40e-6, 80e-6)


def hall_petch_workload(n: int = 32, n_grains: int = 100, strain_max: float = 0.05, n_inc: int = 50,
                        materials=HALL_PETCH_MATERIALS, sizes=HALL_PETCH_SIZES, seed: int = 107):
    """The grain-size study of Section 3: for each material (workload elastic constants, Table 2
    dislocation parameters, the annealed initial density 1e11 per system, i.e. rho_i = 1.2e12),
    one periodic RVE of n^3 voxels with n_grains equiaxed lognormal grains (sd 20 % of the mean)
    scaled to the mean equivalent diameters in sizes (the voxel size follows), plus its twin
    without the GND term (c_gnd = 0, the paper's "infinite" grain size, whose response does not
    depend on the size).  Tension to strain_max in n_inc increments at 1e-4/s.  Returns (RVEs,
    load path, labels (material, size or None for the twin))."""
    gid, _, _ = lognormal_grains(seed, (n, n, n), n_grains)
    d_vox = float(np.mean(equivalent_diameters(gid, n_grains)))
    rves, labels = [], []
    for m_i, name in enumerate(materials):
        quats = shoemake_quaternions(SplitMix64(seed + 1000 + m_i), n_grains)
        for D in list(sizes) + [None]:
            mat = material(name, rho0=1e11, c_gnd=0.0 if D is None else 1.0)
            h = (sizes[0] if D is None else D) / d_vox
            rves.append(RVE(n=(n, n, n), voxel_size=h, grain_of_voxel=gid, quats=quats, material=mat, seed=seed))
            labels.append((name, D))
    return rves, uniaxial_tension(strain_max, n_inc, 1e-4), labels


def beam_cell(n_beam: int = 200, n_clamp: int = 16, n_depth: int = 10, n_soft: int = 10, length: float = 10.0,
              E: float = 200e9, soft: float = 1e-4, clamp: float = 100.0, nz: int = 1):
    """The elastic beam benchmark of Appendix B as a periodic cell (x along the beam, y across):
    a beam of length L = `length` and depth L / 20 (n_beam x n_depth voxels), clamped at both
    ends by a stiff column (n_clamp voxels wide, the whole height) and bounded above and below by
    soft layers of n_soft voxels each, which stand in for free surfaces.  Three isotropic phases
    with Poisson ratio 0 (C11 = E, C12 = 0, C44 = E / 2; with no Poisson coupling the plane-stress
    and plane-strain answers coincide): grain 0 the clamp (clamp x E), grain 1 the beam (E),
    grain 2 the soft layers (soft x E).  Elastic: tau0 = 1e20 Pa and no hardening, so no slip.
    The soft layers stand in for free surfaces only while their shear energy is small against
    the beam's bending energy, whose stiffness scales as (depth / L)^3: at soft = 1e-3 they
    take about twice the bending energy of an L/20 beam and flatten it (curvature 9 % low), at
    1e-4 the effect is near 1 %.
    The load shears the cell by F_21 = delta / L_cell, which moves one clamp by delta = L / 1000
    against the other (beam ends held parallel); F_12 = F_13 = F_23 = F_31 = F_32 = 0 and F_33 = 1
    are prescribed (with F_12 free the cell would rotate instead of bending the beam) and
    P_11 = P_22 = 0.  Returns (RVE, one-increment load path, geometry)."""
    nx, ny = n_clamp + n_beam, 2 * n_soft + n_depth
    h = length / n_beam
    gid = np.full((nz, ny, nx), 2, dtype=np.int32)
    gid[:, n_soft:n_soft + n_depth, :] = 1
    gid[:, :, :n_clamp] = 0
    ge = np.array([[clamp * E, 0.0, clamp * E / 2], [E, 0.0, E / 2], [soft * E, 0.0, soft * E / 2]])
    mat = Material(C11=E, C12=0.0, C44=E / 2, burgers=2.5e-10, y_c=1.5e-8, K_sim=6.0, tau0=1e20, c_gnd=0.0,
                   hardening=0)
    quats = np.tile([1.0, 0.0, 0.0, 0.0], (3, 1))
    rve = RVE(n=(nx, ny, nz), voxel_size=h, grain_of_voxel=gid, quats=quats, material=mat, seed=0,
              grain_elastic=ge)
    delta = length / 1000.0
    F = np.tile(np.eye(3).reshape(9), (2, 1))
    F[1, 3] = delta / (nx * h)
    mask = np.array([0, 1, 1, 1, 0, 1, 1, 1, 1], dtype=np.uint8)
    path = LoadPath(F_bar=F, P_bar=np.zeros((2, 9)), mask=mask, dt=1.0)
    geom = {"n_clamp": n_clamp, "n_beam": n_beam, "n_depth": n_depth, "n_soft": n_soft, "h": h,
            "length": length, "delta": delta}
    return rve, path, geom


def random_deformations(seed: int, count: int, amplitude: float) -> np.ndarray:
    """count near-identity deformation gradients I + amplitude * U(-1, 1), row-major (count, 9)."""
    rng = SplitMix64(seed)
    u = rng.uniforms(9 * count).reshape(count, 9)
    return np.eye(3).reshape(1, 9) + amplitude * (2.0 * u - 1.0)


def random_field(seed: int, shape, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Uniform random array from SplitMix64 (vectorised through numpy for size)."""
    rng = SplitMix64(seed)
    n = int(np.prod(shape))
    # draw 64-bit words in bulk: numpy reproduction of SplitMix64 on a counter
    base = (rng.state + 0x9E3779B97F4A7C15 * (np.arange(1, n + 1, dtype=np.uint64))).astype(np.uint64)
    with np.errstate(over="ignore"):
        z = base
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return (lo + (hi - lo) * u).reshape(shape)


def gaussian_noise(seed: int, n: int) -> np.ndarray:
    """n standard normal draws: Box-Muller (1958) on pairs of SplitMix64 uniforms, the first
    uniform shifted to (0, 1] so that its logarithm is finite."""
    rng = SplitMix64(seed)
    out = np.empty(n)
    for i in range(0, n, 2):
        u1 = 1.0 - rng.uniform()
        u2 = rng.uniform()
        r = math.sqrt(-2.0 * math.log(u1))
        out[i] = r * math.cos(2.0 * math.pi * u2)
        if i + 1 < n:
            out[i + 1] = r * math.sin(2.0 * math.pi * u2)
    return out


# Parameters of the adjoint form: the initial critical stress tau0 (it sets the uniform
# initial SSD density (tau0 / (mu b))^2 / sum_b q^{ab}), the similitude coefficient K of
# eq. 9, the annihilation distance y_c of eq. 8 and the GND weight c_gnd of eqs. 7 and 9.
ADJOINT_PARAMS = ("tau0", "K_sim", "y_c", "c_gnd")


def with_params(mat: Material, theta) -> Material:
    """The material with (tau0, K, y_c, c_gnd) = theta; the initial density then follows tau0."""
    t = [float(v) for v in theta]
    return mat.replace(tau0=t[0], rho0=0.0, K_sim=t[1], y_c=t[2], c_gnd=t[3])


def adjoint_workload(n_override=None, n_inc_override=None):
    """The 64^3 adjoint workload: 100 Voronoi grains (seed 105), Cu, c_gnd = 1, d = 30 um,
    tension to 4 % in 40 increments at 1e-4/s.  The initial state is given by tau0 = 3.47 MPa
    (the critical stress of the annealed density of about 1e11 per system), so that tau0 is one
    of the differentiated parameters.  Returns (rve, path, theta) with theta = (tau0, K, y_c,
    c_gnd)."""
    rves, path = workload("cu64g100", n_override=n_override)
    rve = rves[0]
    mat = rve.material
    theta = (3.47e6, mat.K_sim, mat.y_c, 1.0)
    rve = dataclasses.replace(rve, material=with_params(mat, theta))
    if n_inc_override:
        path = LoadPath(F_bar=path.F_bar[: n_inc_override + 1], P_bar=path.P_bar[: n_inc_override + 1],
                        mask=path.mask, dt=path.dt)
    return rve, path, theta
