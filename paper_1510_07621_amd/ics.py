"""Seeded synthetic particle sets and the named workloads built from them.

This module only draws inputs. It holds none of the force method's
arithmetic, so both the GPU path's tests and the CPU reference can take
their particles from here.

Layout follows the guide's particle container (CONCEPT User's Guide,
Ch. 6 "Snapshot Formats", standard format): one mass per particle group and
structure-of-arrays comoving positions, here a C-contiguous float64 array of
shape (3, N) holding x, y and z rows, each component in [0, box).

Recipes (the guide gives none; these are stated readings):

* ``uniform``: N points uniform in the periodic cube.
* ``zeldovich_lattice``: a cubic lattice q = i*s displaced by a Gaussian random
  field with power spectrum P(k) proportional to k^-2. White noise w is
  transformed, multiplied by k^-1 (so |delta_k|^2 ~ k^-2), the k = 0 mode and
  every Nyquist index are zeroed, the displacement is psi_k = i k delta_k / k^2
  (so div psi = -delta), and psi is scaled so that the 3-D vector rms of
  |psi| equals ``rms_frac`` times the lattice spacing s.
* ``plummer_mix``: a fraction of the particles in Plummer spheres with
  uniformly placed centres and log-uniform scale radii. Each clustered
  particle picks a sphere uniformly at random (so sphere masses follow the
  multinomial counts). Radii follow the Plummer cumulative mass profile
  truncated at ten scale radii, r = a (u^(-2/3) - 1)^(-1/2) with
  u ~ U(0, 1000/101^1.5); directions are isotropic. The rest is uniform.

All generators use ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "uniform",
    "zeldovich_lattice",
    "plummer_mix",
    "lattice",
    "wrap_positions",
    "Workload",
    "WORKLOADS",
    "workload",
]


def wrap_positions(x: np.ndarray, box: float) -> np.ndarray:
    """Map coordinates into [0, box) (a value that rounds to box becomes 0)."""
    y = np.mod(x, box)
    y[y >= box] = 0.0
    return y


def uniform(n: int, box: float = 1.0, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    pos = rng.random((3, n)) * box
    return wrap_positions(pos, box)


def lattice(n_side: int, box: float = 1.0, offset: float = 0.0) -> np.ndarray:
    """Simple cubic lattice, n_side^3 points at (i + offset) * box / n_side."""
    s = box / n_side
    g = (np.arange(n_side, dtype=np.float64) + offset) * s
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()]))


def zeldovich_lattice(n_side: int, box: float = 1.0, seed: int = 2,
                      rms_frac: float = 0.3, return_parts: bool = False):
    """Lattice plus a P(k) ~ k^-2 Gaussian-random-field displacement.

    Returns positions (3, N); with ``return_parts`` also (q, psi) such that
    positions = wrap(q + psi)."""
    rng = np.random.default_rng(seed)
    n = n_side
    s = box / n
    w = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(w)
    fx = np.fft.fftfreq(n, d=1.0 / n)          # integer wavenumbers
    fz = np.fft.rfftfreq(n, d=1.0 / n)
    kx = (2 * np.pi / box) * fx[:, None, None]
    ky = (2 * np.pi / box) * fx[None, :, None]
    kz = (2 * np.pi / box) * fz[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    delta_k = wk / np.sqrt(k2)
    delta_k[0, 0, 0] = 0.0
    if n % 2 == 0:
        nyq = n // 2
        delta_k[nyq, :, :] = 0.0
        delta_k[:, nyq, :] = 0.0
        delta_k[:, :, nyq] = 0.0
    psi = np.empty((3, n, n, n))
    for d, kd in enumerate((kx, ky, kz)):
        psi[d] = np.fft.irfftn(1j * kd * delta_k / k2, s=(n, n, n), axes=(0, 1, 2))
    rms = math.sqrt(float(np.mean(np.sum(psi * psi, axis=0))))
    psi *= rms_frac * s / rms
    q = lattice(n, box)
    psi = np.ascontiguousarray(psi.reshape(3, -1))
    pos = wrap_positions(q + psi, box)
    if return_parts:
        return pos, q, psi
    return pos


PLUMMER_U_MAX = 1000.0 / 101.0 ** 1.5   # Plummer mass fraction inside 10 scale radii


def plummer_mix(n: int, box: float = 1.0, seed: int = 3, n_spheres: int = 2000,
                frac: float = 0.7, a_min: float = 0.002, a_max: float = 0.02,
                return_labels: bool = False):
    """70 % of particles in Plummer spheres, 30 % uniform background (defaults).

    With ``return_labels`` also returns the sphere index of each particle
    (-1 for the background), the centres and the scale radii."""
    rng = np.random.default_rng(seed)
    centres = rng.random((n_spheres, 3)) * box
    a = np.exp(rng.uniform(math.log(a_min), math.log(a_max), n_spheres)) * box
    n_cl = int(round(frac * n))
    which = rng.integers(0, n_spheres, n_cl)
    u = rng.uniform(0.0, PLUMMER_U_MAX, n_cl)
    r = a[which] * (u ** (-2.0 / 3.0) - 1.0) ** -0.5
    v = rng.standard_normal((n_cl, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    cl = centres[which] + r[:, None] * v
    bg = rng.random((n - n_cl, 3)) * box
    pos = np.ascontiguousarray(np.concatenate([cl, bg]).T)
    pos = wrap_positions(pos, box)
    if return_labels:
        labels = np.concatenate([which, -np.ones(n - n_cl, dtype=which.dtype)])
        return pos, labels, centres, a
    return pos


@dataclasses.dataclass(frozen=True)
class Workload:
    """A named force-evaluation workload: particles plus the P3M parameters.

    ``rs_cells`` is the split scale in PM cells and ``cutoff_rs`` the
    short-range cutoff in split scales (guide Ch. 5, PM_scale and
    P3M_cutoff); ``soft_frac`` is the Plummer radius in mean inter-particle
    spacings (guide Ch. 5, softeningfactors)."""
    name: str
    n_side: int
    grid_n: int
    recipe: str
    seed: int
    box: float = 1.0
    rs_cells: float = 1.25
    cutoff_rs: float = 4.5
    soft_frac: float = 0.03
    G: float = 1.0
    steps: int = 0
    dt: float = 0.0

    @property
    def n(self) -> int:
        return self.n_side ** 3

    @property
    def h(self) -> float:
        return self.box / self.grid_n

    @property
    def r_s(self) -> float:
        return self.rs_cells * self.h

    @property
    def r_c(self) -> float:
        return self.cutoff_rs * self.r_s

    @property
    def softening(self) -> float:
        return self.soft_frac * self.box / self.n_side

    @property
    def mass(self) -> float:
        """Equal masses summing to one, so the mean density is 1/box^3."""
        return 1.0 / self.n

    def positions(self) -> np.ndarray:
        if self.recipe == "uniform":
            return uniform(self.n, self.box, self.seed)
        if self.recipe == "zeldovich":
            return zeldovich_lattice(self.n_side, self.box, self.seed)
        if self.recipe == "plummer":
            return plummer_mix(self.n, self.box, self.seed)
        raise ValueError(self.recipe)

    def params(self) -> dict:
        return dict(grid_n=self.grid_n, box=self.box, rs_cells=self.rs_cells,
                    cutoff_rs=self.cutoff_rs, softening=self.softening, G=self.G)


WORKLOADS = {
    # 32^3 uniform random particles, 32^3 grid, FP64: the small accuracy case.
    "uniform32": Workload("uniform32", 32, 32, "uniform", seed=1),
    # 128^3 Zel'dovich-displaced lattice (P(k) ~ k^-2, rms 0.3 spacing), 128^3 grid.
    "zeldovich128": Workload("zeldovich128", 128, 128, "zeldovich", seed=2),
    # 256^3 particles, 70 % in 2000 Plummer spheres, 256^3 grid.
    "plummer256": Workload("plummer256", 256, 256, "plummer", seed=3),
    # 64^3 Zel'dovich ICs, 64^3 grid, 10 leapfrog steps of dt = 0.01.
    "zeldovich64_kdk": Workload("zeldovich64_kdk", 64, 64, "zeldovich", seed=4,
                                steps=10, dt=0.01),
    # 128^3 Plummer mix, 128^3 grid, 50 leapfrog steps of dt = 0.001: the
    # smallest spheres (a = 0.002 box, ~734 particles) have a dynamical time
    # sqrt(a^3 / (G M)) ~ 5e-3, which a step of 0.01 would not resolve.
    "plummer128_kdk": Workload("plummer128_kdk", 128, 128, "plummer", seed=5,
                               steps=50, dt=0.001),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]
