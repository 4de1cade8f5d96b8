"""Voxel discretisation of a disk or sphere meta-atom (oracle, FP64).

The paper discretises the polarisation current with loop/star functions on a
tetrahedral mesh (§3, eq. 3.1).  The configured workloads instead voxelise each
disk into 48 cells with three Cartesian current components per cell; this module
is the oracle's reading of that rule:

* 24 in-plane squares of side h = r * sqrt(pi / 24): the squares of the
  h-grid whose centres ((a + 1/2) h, (b + 1/2) h) satisfy
  (a + 1/2)^2 + (b + 1/2)^2 <= 24 / pi, i.e. the offset classes
  (+-1/2, +-1/2), (+-1/2, +-3/2), (+-3/2, +-1/2), (+-3/2, +-3/2),
  (+-1/2, +-5/2), (+-5/2, +-1/2): 4 + 8 + 4 + 8 = 24 squares;
* two layers of thickness t / 2 centred at z = -t/4 and z = +t/4;
* cell volume V = h^2 t / 2, so 48 V = pi r^2 t (volume-exact);
* canonical order: layer (lower, upper), then b ascending, then a ascending;
  DoF index = (cell * 3 + component), component x, y, z fastest.

Spheres (``sphere_cells``): 48 equal cubes, four layers of a 4 x 4 grid without corners.

Pins (tests): 24 squares, volume exactness, symmetry of the offset set; the
equal-volume sphere radius of a cell in closed form, (r^2 t / 64)^(1/3); for spheres,
48 distinct non-overlapping cubes whose volume is the sphere's, mirror symmetry in x, y, z.
Unknowns are ordered particle by particle (§4, eq. 4.1).
"""
from __future__ import annotations

import math

import numpy as np

N_SQUARES = 24
N_CELLS = 48
N_DOF_PER_PARTICLE = N_CELLS * 3


def square_offsets() -> np.ndarray:
    """(24, 2) in-plane square centres in units of h, canonical (b, a) order."""
    out = []
    limit = 24.0 / math.pi
    for b in range(-3, 3):
        for a in range(-3, 3):
            cx, cy = a + 0.5, b + 0.5
            if cx * cx + cy * cy <= limit:
                out.append((cx, cy))
    arr = np.array(out, dtype=np.float64)
    assert arr.shape == (N_SQUARES, 2), arr.shape
    return arr


def particle_cells(radius: float, height: float) -> tuple[np.ndarray, float]:
    """Cell-centre offsets (48, 3) relative to the particle centre, and the cell volume."""
    h = radius * math.sqrt(math.pi / 24.0)
    sq = square_offsets() * h
    cells = np.zeros((N_CELLS, 3), dtype=np.float64)
    for layer, z in enumerate((-height / 4.0, height / 4.0)):
        cells[layer * N_SQUARES:(layer + 1) * N_SQUARES, 0:2] = sq
        cells[layer * N_SQUARES:(layer + 1) * N_SQUARES, 2] = z
    vol = h * h * height / 2.0
    return cells, vol


def sphere_cells(radius: float) -> tuple[np.ndarray, float]:
    """Voxelised sphere (the paper's meta-atom, §6.1; shape-only stand-in for its mesh):
    48 cubes of side h with 48 h^3 = (4/3) pi r^3, i.e. h = r (pi/36)^(1/3), in four layers
    z in {-3/2, -1/2, 1/2, 3/2} h; each layer holds the cubes of a 4 x 4 grid of centres
    (x, y) in {-3/2, -1/2, 1/2, 3/2} h except the four with |x| = |y| = 3h/2.
    Canonical order: layer, then y ascending, then x ascending."""
    h = radius * (math.pi / 36.0) ** (1.0 / 3.0)
    ticks = (-1.5, -0.5, 0.5, 1.5)
    out = []
    for z in ticks:
        for y in ticks:
            for x in ticks:
                if abs(x) == 1.5 and abs(y) == 1.5:
                    continue
                out.append((x * h, y * h, z * h))
    cells = np.array(out, dtype=np.float64)
    assert cells.shape == (N_CELLS, 3)
    return cells, h ** 3


def equivalent_radius(volume: float) -> float:
    """Radius of the sphere with the cell's volume (used by the self term)."""
    return (3.0 * volume / (4.0 * math.pi)) ** (1.0 / 3.0)


class Discretisation:
    """All cells of an array, particle-major in caller order."""

    def __init__(self, array):
        n = array.n_particles
        self.n_particles = n
        self.k = 2.0 * math.pi / array.wavelength
        self.offsets = np.zeros((n, N_CELLS, 3))
        self.pos = np.zeros((n, N_CELLS, 3))
        self.vol = np.zeros(n)
        self.a_eq = np.zeros(n)
        self.chi = np.asarray(array.eps_r, dtype=np.complex128) - 1.0
        sphere = getattr(array, "shape", "disk") == "sphere"
        for p in range(n):
            if sphere:
                off, v = sphere_cells(float(array.radius[p]))
            else:
                off, v = particle_cells(float(array.radius[p]), float(array.height[p]))
            self.offsets[p] = off
            self.pos[p] = array.centers[p][None, :] + off
            self.vol[p] = v
            self.a_eq[p] = equivalent_radius(v)

    @property
    def ndof(self) -> int:
        return self.n_particles * N_DOF_PER_PARTICLE

    def cell_arrays(self):
        """Flattened per-cell position (nc, 3), volume (nc,), chi (nc,), a_eq (nc,)."""
        pos = self.pos.reshape(-1, 3)
        vol = np.repeat(self.vol, N_CELLS)
        chi = np.repeat(self.chi, N_CELLS)
        aeq = np.repeat(self.a_eq, N_CELLS)
        return pos, vol, chi, aeq
