"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module describes *inputs only*: particle centres on a rectangular lattice,
per-particle radius, height and relative permittivity, plane-wave incidences and
the request stream of the serving workload.  It holds none of the method's
arithmetic (no discretisation, no Green's function, no grouping, no solver), so
the oracle and the HIP library can both take their inputs from here and still
share no code.

Units: lengths in free-space wavelengths (wavelength = 1).

Workload recipes (the array sizes and distributions below follow the configured
workloads; the paper's own test geometry, a Vogel spiral of spheres, is given by
``vogel_centers``):

* tiny      4x4 lattice, pitch 0.5, all radii 0.2, height 0.1, eps_r 12+0.1i
* mid       32x32 lattice, radii U[0.15, 0.25] from ``default_rng(0)``
* batching  64x64 lattice, graded metalens radius profile (``graded_metalens_radii``)
* precision 96x96 lattice, radii U[0.15, 0.25] from ``default_rng(0)``
* serving   256 requests, side U{8..48}, radii U[0.15, 0.25], 1-16 RHS, Poisson arrivals
* vogel     the paper's arrays: n = 100 / 500 / 1000 / 2000 gold spheres (radius 1/6) on a
            Vogel spiral, grouped on the paper's grid
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

EPS_R_DEFAULT = 12.0 + 0.1j
PITCH_DEFAULT = 0.5
HEIGHT_DEFAULT = 0.1
CELLS_PER_PARTICLE = 48


@dataclass
class ArrayDesc:
    """A lattice array of disks, in caller order p = j * nx + i."""

    nx: int
    ny: int
    pitch: float
    centers: np.ndarray          # (N, 3) float64
    lattice_ij: np.ndarray       # (N, 2) int32, (i, j) lattice indices
    radius: np.ndarray           # (N,) float64
    height: np.ndarray           # (N,) float64
    eps_r: np.ndarray            # (N,) complex128
    wavelength: float = 1.0
    cells_per_particle: int = CELLS_PER_PARTICLE
    name: str = ""
    shape: str = "disk"          # "disk" or "sphere"
    grid: str = "lattice"        # "lattice" (lattice_ij) or "paper" (blocks from the centres)

    @property
    def n_particles(self) -> int:
        return int(self.centers.shape[0])

    @property
    def ndof(self) -> int:
        return self.n_particles * self.cells_per_particle * 3


def lattice(nx: int, ny: int | None = None, *, pitch: float = PITCH_DEFAULT,
            radius=0.2, height=HEIGHT_DEFAULT, eps_r=EPS_R_DEFAULT,
            name: str = "") -> ArrayDesc:
    """nx x ny lattice centred on the origin in the z = 0 plane."""
    ny = nx if ny is None else ny
    n = nx * ny
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = ii.reshape(-1).astype(np.int32)
    j = jj.reshape(-1).astype(np.int32)
    centers = np.zeros((n, 3), dtype=np.float64)
    centers[:, 0] = (i - (nx - 1) / 2.0) * pitch
    centers[:, 1] = (j - (ny - 1) / 2.0) * pitch
    rad = np.broadcast_to(np.asarray(radius, dtype=np.float64), (n,)).copy()
    hgt = np.broadcast_to(np.asarray(height, dtype=np.float64), (n,)).copy()
    eps = np.broadcast_to(np.asarray(eps_r, dtype=np.complex128), (n,)).copy()
    return ArrayDesc(nx=nx, ny=ny, pitch=pitch, centers=centers,
                     lattice_ij=np.stack([i, j], axis=1).astype(np.int32),
                     radius=rad, height=hgt, eps_r=eps, name=name)


def uniform_radii(n: int, seed: int, lo: float = 0.15, hi: float = 0.25) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


def graded_metalens_radii(nx: int, ny: int, pitch: float = PITCH_DEFAULT) -> np.ndarray:
    """r(x, y) = 0.15 + 0.1 * frac(phi / 2pi), phi = pi rho^2 / F, F = side * pitch."""
    d = lattice(nx, ny, pitch=pitch)
    rho2 = d.centers[:, 0] ** 2 + d.centers[:, 1] ** 2
    focal = max(nx, ny) * pitch
    phase = math.pi * rho2 / focal
    frac = np.mod(phase / (2.0 * math.pi), 1.0)
    return 0.15 + 0.1 * frac


def tiny() -> ArrayDesc:
    return lattice(4, radius=0.2, name="tiny-4x4")


def mid(seed: int = 0) -> ArrayDesc:
    return lattice(32, radius=uniform_radii(32 * 32, seed), name="mid-32x32")


def random_lattice(nx: int, ny: int | None = None, seed: int = 0) -> ArrayDesc:
    ny = nx if ny is None else ny
    return lattice(nx, ny, radius=uniform_radii(nx * ny, seed), name=f"rand-{nx}x{ny}-s{seed}")


def batching() -> ArrayDesc:
    return lattice(64, radius=graded_metalens_radii(64, 64), name="batching-64x64")


def precision(seed: int = 0) -> ArrayDesc:
    return lattice(96, radius=uniform_radii(96 * 96, seed), name="precision-96x96")


# ---------------------------------------------------------------- incidences
TE, TM = 0, 1


@dataclass
class Incidence:
    theta_deg: np.ndarray
    phi_deg: np.ndarray
    pol: np.ndarray   # int32, 0 = TE, 1 = TM

    @property
    def nrhs(self) -> int:
        return int(self.theta_deg.shape[0])


def normal_x() -> Incidence:
    """Normal incidence, x-polarised (theta = 0, phi = 0, TM)."""
    return Incidence(np.array([0.0]), np.array([0.0]), np.array([TM], dtype=np.int32))


def mid_incidence() -> Incidence:
    return Incidence(np.array([10.0]), np.array([0.0]), np.array([TM], dtype=np.int32))


def sweep(n_theta: int, lo: float = -30.0, hi: float = 30.0) -> Incidence:
    th = np.linspace(lo, hi, n_theta)
    theta = np.concatenate([th, th])
    pol = np.concatenate([np.full(n_theta, TE), np.full(n_theta, TM)]).astype(np.int32)
    return Incidence(theta, np.zeros_like(theta), pol)


def random_incidence(nrhs: int, rng: np.random.Generator) -> Incidence:
    theta = rng.uniform(-30.0, 30.0, nrhs)
    pol = rng.integers(0, 2, nrhs).astype(np.int32)
    return Incidence(theta, np.zeros(nrhs), pol)


# ---------------------------------------------------------------- serving
@dataclass
class Request:
    rid: int
    arrival_s: float
    array: ArrayDesc
    incidence: Incidence
    tol: float = 1e-6


def serving_requests(n: int = 256, seed: int = 0, rate_per_s: float = 1.0,
                     side_lo: int = 8, side_hi: int = 48) -> list[Request]:
    """Poisson arrivals; side U{side_lo..side_hi}; radii U[0.15, 0.25]; 1-16 RHS."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        side = int(rng.integers(side_lo, side_hi + 1))
        radii = rng.uniform(0.15, 0.25, side * side)
        nrhs = int(rng.integers(1, 17))
        inc = random_incidence(nrhs, rng)
        arr = lattice(side, radius=radii, name=f"req{rid}-{side}x{side}")
        out.append(Request(rid=rid, arrival_s=t, array=arr, incidence=inc))
    return out


# ---------------------------------------------------------------- Vogel spiral
def vogel_centers(n: int, sphere_radius: float) -> np.ndarray:
    """Vogel spiral (paper §6.1): r_i = c sqrt(i), c = R sqrt(3), angle i * golden angle.

    The golden ratio is (1 + sqrt 5) / 2 (the printed formula misplaces a
    parenthesis); the golden angle is 2 pi / phi^2.
    """
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    alpha = 2.0 * math.pi / phi ** 2
    c = sphere_radius * math.sqrt(3.0)
    i = np.arange(1, n + 1, dtype=np.float64)
    r = c * np.sqrt(i)
    return np.stack([r * np.cos(i * alpha), r * np.sin(i * alpha), np.zeros(n)], axis=1)


VOGEL_SPHERE_RADIUS = 0.1 / 0.6          # 100 nm spheres at 600 nm wavelength
VOGEL_EPS_R = -9.428 - 1.513j             # gold at 500 THz, passive sign for the e^{+j omega t} convention


def vogel(n: int) -> ArrayDesc:
    """The paper's test array (§6.1): n gold spheres of radius 100 nm on a Vogel spiral at a
    600 nm wavelength, grouped on the paper's grid (no lattice).  The tabulated permittivity
    -9.428 + 1.513i belongs to the e^{-i omega t} convention; with the e^{+j omega t}
    convention of the kernel the same passive (lossy) gold is -9.428 - 1.513j."""
    centers = vogel_centers(n, VOGEL_SPHERE_RADIUS)
    r = np.full(n, VOGEL_SPHERE_RADIUS)
    return ArrayDesc(nx=0, ny=0, pitch=0.0, centers=centers, lattice_ij=np.zeros((n, 2), dtype=np.int32),
                     radius=r, height=2.0 * r, eps_r=np.full(n, VOGEL_EPS_R, dtype=np.complex128),
                     name=f"vogel-{n}", shape="sphere", grid="paper")


def to_c_desc_arrays(a: ArrayDesc) -> dict:
    """Flat, C-contiguous arrays in the layout the C ABI takes."""
    return dict(
        n=a.n_particles,
        centers=np.ascontiguousarray(a.centers, dtype=np.float64),
        radius=np.ascontiguousarray(a.radius, dtype=np.float64),
        height=np.ascontiguousarray(a.height, dtype=np.float64),
        eps_r=np.ascontiguousarray(a.eps_r, dtype=np.complex128),
        lattice_ij=np.ascontiguousarray(a.lattice_ij, dtype=np.int32),
        pitch=float(a.pitch), wavelength=float(a.wavelength),
        cells_per_particle=int(a.cells_per_particle),
    )
