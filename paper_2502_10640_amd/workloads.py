"""Seeded synthetic bunch generators shared by the oracle checks, the GPU tests
and the benchmark.

This module holds input generation only: particle placement, thermal
velocities, per-particle charge and mass arrays, and the setup arithmetic that
turns a physical description (radius, total charge, temperature, time step in
units of the plasma period) into numbers.  It contains none of the method's
arithmetic (no field, no push, no diagnostics), imports nothing from the HIP
binding and nothing from the oracle.

Physical setting (arXiv 2502.10640, Sec. 2.1): an electron bunch made of N_p
macro-particles, each standing for w_p real electrons (all macro-particles share
one weight), expanding in vacuum from a given spatial and velocity
distribution.  The paper's own bunch is a cubic lattice (Sec. 2.1 setup
paragraph); the benchmark workloads are seeded spheres and Gaussians.

Readings of points the paper does not fix:
  * mean spacing = (V / N_p)^(1/3), with V = 4 pi R^3 / 3 for a sphere and
    V = (2 pi)^(3/2) sx sy sz for a Gaussian (peak-density volume);
  * plasma frequency omega_p = sqrt(n_e e^2 / (eps0 m_e)), n_e = electrons / V;
  * uniform sphere: radius R u^(1/3) along a normalised Gaussian direction;
    Gaussian bunch: N(0, sigma^2) per axis; Maxwellian: N(0, kT/m_e) per
    velocity component; positions and velocities are then shifted to zero
    mean (centre-of-mass frame, zero momentum);
  * cube lattice: cell-centred points x_k = (k + 1/2) l/n - l/2.
Random numbers come from NumPy's PCG64 ``default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

# CODATA 2018 values.
E_CHARGE = 1.602176634e-19      # C (exact)
M_ELECTRON = 9.1093837015e-31   # kg
EPS0 = 8.8541878128e-12         # F/m
EV = E_CHARGE                   # J per eV


@dataclass
class Bunch:
    """One bunch: FP64 SoA arrays and its per-bunch scalars (SI units)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    q: np.ndarray        # real-particle charge per macro-particle [C]
    m: np.ndarray        # real-particle mass per macro-particle [kg]
    weight: float        # real particles per macro-particle
    softening: float     # Plummer length [m]
    dt: float            # time step [s]
    n_steps: int = 0     # steps the workload asks for
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return (self.x, self.y, self.z, self.vx, self.vy, self.vz, self.q, self.m)

    def copy(self) -> "Bunch":
        return Bunch(*(a.copy() for a in self.arrays()), self.weight, self.softening,
                     self.dt, self.n_steps, dict(self.meta))


# ----------------------------------------------------------------------------
# placement and velocities
# ----------------------------------------------------------------------------

def sphere_uniform(n: int, radius: float, rng: np.random.Generator):
    """n points uniform in a ball of the given radius."""
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    p = d * r[:, None]
    return p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()


def gaussian(n: int, sigma, rng: np.random.Generator):
    """n points with independent N(0, sigma_a^2) coordinates."""
    s = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (3,))
    p = rng.standard_normal((n, 3)) * s[None, :]
    return p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()


def maxwellian(n: int, temperature_ev: float, rng: np.random.Generator, mass=M_ELECTRON):
    """n velocities with N(0, kT/m) components."""
    sv = math.sqrt(temperature_ev * EV / mass)
    v = rng.standard_normal((n, 3)) * sv
    return v[:, 0].copy(), v[:, 1].copy(), v[:, 2].copy()


def cube_lattice(n_side: int, side: float):
    """Cell-centred cubic lattice of n_side^3 points in a cube of the given side."""
    c = (np.arange(n_side) + 0.5) * side / n_side - side / 2.0
    gx, gy, gz = np.meshgrid(c, c, c, indexing="ij")
    return gx.ravel().copy(), gy.ravel().copy(), gz.ravel().copy()


def zero_mean(*arrays):
    """Shift each array to zero mean (centre-of-mass frame for equal masses)."""
    return tuple(a - a.mean() for a in arrays)


# ----------------------------------------------------------------------------
# setup arithmetic
# ----------------------------------------------------------------------------

def sphere_volume(radius: float) -> float:
    return 4.0 * math.pi * radius ** 3 / 3.0


def gaussian_volume(sigma) -> float:
    s = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (3,))
    return (2.0 * math.pi) ** 1.5 * float(s[0] * s[1] * s[2])


def mean_spacing(n: int, volume: float) -> float:
    return (volume / n) ** (1.0 / 3.0)


def plasma_frequency(n_e: float) -> float:
    """omega_p [rad/s] of an electron density n_e [1/m^3]."""
    return math.sqrt(n_e * E_CHARGE ** 2 / (EPS0 * M_ELECTRON))


def electron_arrays(n: int):
    """q = -e and m = m_e for every macro-particle (Sec. 2.1, Eqs. (E)/(F))."""
    return np.full(n, -E_CHARGE), np.full(n, M_ELECTRON)


def _bunch(x, y, z, vx, vy, vz, electrons_total, softening, dt, n_steps, meta) -> Bunch:
    n = x.shape[0]
    q, m = electron_arrays(n)
    return Bunch(x, y, z, vx, vy, vz, q, m, electrons_total / n, softening, dt, n_steps, meta)


def cold_sphere(n: int, radius: float, electrons_total: float, eps_frac: float, dt_omega: float,
                n_steps: int, seed: int, name: str = "cold_sphere") -> Bunch:
    """Uniform sphere at rest: eps = eps_frac x mean spacing, dt = dt_omega / omega_p."""
    rng = np.random.default_rng(seed)
    x, y, z = zero_mean(*sphere_uniform(n, radius, rng))
    vol = sphere_volume(radius)
    wp = plasma_frequency(electrons_total / vol)
    spacing = mean_spacing(n, vol)
    zeros = np.zeros(n)
    meta = dict(name=name, geometry="sphere", radius=radius, electrons=electrons_total,
                omega_p=wp, spacing=spacing, seed=seed, dt_omega=dt_omega)
    return _bunch(x, y, z, zeros.copy(), zeros.copy(), zeros.copy(), electrons_total,
                  eps_frac * spacing, dt_omega / wp, n_steps, meta)


def gaussian_bunch(n: int, sigma, temperature_ev: float, electrons_total: float, eps_frac: float,
                   dt_omega: float, n_steps: int, seed: int, name: str = "gaussian") -> Bunch:
    """Gaussian bunch with Maxwellian velocities; density and spacing at the peak."""
    rng = np.random.default_rng(seed)
    x, y, z = zero_mean(*gaussian(n, sigma, rng))
    vx, vy, vz = zero_mean(*maxwellian(n, temperature_ev, rng))
    vol = gaussian_volume(sigma)
    wp = plasma_frequency(electrons_total / vol)
    spacing = mean_spacing(n, vol)
    meta = dict(name=name, geometry="gaussian", sigma=list(np.broadcast_to(sigma, (3,)).astype(float)),
                temperature_ev=temperature_ev, electrons=electrons_total, omega_p=wp,
                spacing=spacing, seed=seed, dt_omega=dt_omega)
    return _bunch(x, y, z, vx, vy, vz, electrons_total, eps_frac * spacing, dt_omega / wp,
                  n_steps, meta)


def paper_cube(n_side: int = 16, side: float = 1e-4, density: float = 5e16, dt: float = 1e-13,
               n_steps: int = 100_000, softening: float = 0.0) -> Bunch:
    """The paper's bunch (Sec. 2.1 setup): cube of side l = 0.1 mm, n0 = 5e16 m^-3,
    n_side^3 macro-particles at rest on a uniform lattice, dt = 1e-13 s."""
    x, y, z = cube_lattice(n_side, side)
    n = x.shape[0]
    zeros = np.zeros(n)
    electrons = density * side ** 3
    meta = dict(name=f"paper_cube_{n_side}^3", geometry="cube", side=side, density=density,
                electrons=electrons, omega_p=plasma_frequency(density), spacing=side / n_side)
    return _bunch(x, y, z, zeros.copy(), zeros.copy(), zeros.copy(), electrons, softening, dt,
                  n_steps, meta)


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

SWEEP_DT = (0.002, 0.005, 0.01, 0.02)


def sweep_sizes(n_bunches: int = 64, lo: int = 4096, hi: int = 131072, seed: int = 1004) -> List[int]:
    rng = np.random.default_rng(seed)
    u = rng.random(n_bunches)
    return [int(round(math.exp(math.log(lo) + ui * (math.log(hi) - math.log(lo))))) for ui in u]


def workload(name: str, n_override: int | None = None) -> List[Bunch]:
    """The named synthetic workloads; returns a list of bunches.

    cold_sphere_2048     uniform sphere R = 100 um, 2 048 particles, 1e8 electrons,
                         eps = 1e-3 spacing, dt = 0.01/omega_p, 100 steps (seed 1001)
    gaussian_65536       Gaussian sigma = 50 um, Maxwellian T = 1 eV, 65 536 particles,
                         1e9 electrons, eps = 1e-3 spacing, dt = 0.01/omega_p, 1000 steps (1002)
    cold_sphere_1m       uniform sphere R = 200 um, 1 048 576 particles, 1e10 electrons,
                         eps = 5e-4 spacing, dt = 0.005/omega_p, 200 steps (1003)
    sweep_64             64 uniform spheres R = 100 um, 1e9 electrons each, sizes
                         log-uniform in [4096, 131072] (1004), dt cycling over
                         {0.002, 0.005, 0.01, 0.02}/omega_p, 500 steps
    ellipsoid_4m         Gaussian sigma = (30, 30, 300) um, T = 0.5 eV, 4 194 304
                         particles, 4e10 electrons, eps = 5e-4 spacing,
                         dt = 0.005/omega_p, 20 steps (1005)
    paper_cube_16        the paper's 16^3 lattice cube (Sec. 2.1), eps = 0
    paper_np_batch       the paper's macro-particle sweep (Sec. 2.2): cubes of 4^3, 8^3,
                         16^3 and 32^3 particles, dt = 1e-13 s, as one batch
    ``n_override`` replaces the particle count (same recipe, smaller or larger).
    """
    if name == "cold_sphere_2048":
        return [cold_sphere(n_override or 2048, 100e-6, 1e8, 1e-3, 0.01, 100, 1001, name)]
    if name == "gaussian_65536":
        return [gaussian_bunch(n_override or 65536, 50e-6, 1.0, 1e9, 1e-3, 0.01, 1000, 1002, name)]
    if name == "cold_sphere_1m":
        return [cold_sphere(n_override or 1048576, 200e-6, 1e10, 5e-4, 0.005, 200, 1003, name)]
    if name == "ellipsoid_4m":
        return [gaussian_bunch(n_override or 4194304, (30e-6, 30e-6, 300e-6), 0.5, 4e10, 5e-4,
                               0.005, 20, 1005, name)]
    if name == "sweep_64":
        sizes = sweep_sizes()
        if n_override:
            sizes = sizes[:max(1, int(n_override))]
        out = []
        for b, nb in enumerate(sizes):
            out.append(cold_sphere(nb, 100e-6, 1e9, 1e-3, SWEEP_DT[b % 4], 500, 1004 * 1000 + b,
                                   f"sweep_64[{b}]"))
        return out
    if name == "paper_cube_16":
        return [paper_cube(16)]
    if name == "paper_np_batch":
        return [paper_cube(k) for k in (4, 8, 16, 32)]
    raise KeyError(name)


WORKLOADS = ("cold_sphere_2048", "gaussian_65536", "cold_sphere_1m", "sweep_64", "ellipsoid_4m",
             "paper_cube_16", "paper_np_batch")


def concat(bunches: List[Bunch]):
    """Flatten bunches into one SoA set plus an offset table (offset, n) per bunch."""
    arrays = [np.concatenate([b.arrays()[k] for b in bunches]) for k in range(8)]
    offsets, off = [], 0
    for b in bunches:
        offsets.append((off, b.n))
        off += b.n
    return arrays, offsets
