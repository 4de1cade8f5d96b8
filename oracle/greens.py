"""Interaction matrix Z and incident field v0 of the voxel VIE (oracle, FP64).

The integral equation of §2 (eq. 2.4) with the scalar Green's function
g(R) = exp(-j k R) / (4 pi R) (time convention exp(+j omega t), §2) is written
for the normalised polarisation p = chi E.  Combining the vector-potential and
charge terms of eq. 2.4 gives the dyadic kernel (I + grad grad / k^2) g:

    G(d) = g(R) [ (1 - j/(kR) - 1/(kR)^2) I + (-1 + 3j/(kR) + 3/(kR)^2) d^ d^T ],
    R = |d|, d^ = d / R.

Galerkin projection on pulse functions with one-point quadrature (the
discretisation reading for the voxel workloads; the symmetric weak form of
eq. 2.5 makes Z complex-symmetric):

    Z[(m,a),(n,b)] = -k^2 V_m V_n G_ab(r_m - r_n)             m != n
    Z[(m,a),(m,b)] = V_m delta_ab [ 1/chi_m - s(a_m) ]
    s(a) = (2/3) [ (1 + j k a) exp(-j k a) - 1 ] - 1/3

s(a) is k^2 times the principal-value integral of G over the sphere of the
cell's volume plus the -1/3 depolarisation; it takes the place of the R and
self parts of L, D in eq. 3.5.  Right-hand side (eq. 3.4, v0):
v[(m,a)] = V_m E0_a(r_m), E0(r) = e exp(-j k k^ . r).

Pins (tests): exact symmetry Z = Z^T; finite-difference check of G against
(I + grad grad / k^2) g; far-field limit G -> g (I - d^ d^); the small-ka series
s(a) = -1/3 + (ka)^2/3 - j (2/9)(ka)^3; the static single-cell
Clausius-Mossotti limit p = 3 (eps - 1)/(eps + 2) E0; oblique TE/TM plane waves equal
the polarisation triad rotated from the z-directed wave; for any p, the imaginary part
of the off-diagonal form plus the point-dipole self radiation equals the power the cell
dipoles radiate (an independent far-field quadrature).
"""
from __future__ import annotations

import math

import numpy as np

from .discretise import N_CELLS, N_DOF_PER_PARTICLE


def scalar_g(R: np.ndarray, k: float) -> np.ndarray:
    return np.exp(-1j * k * R) / (4.0 * math.pi * R)


def dyadic(d: np.ndarray, k: float) -> np.ndarray:
    """Dyadic Green's function for separation vectors d (..., 3) -> (..., 3, 3)."""
    d = np.asarray(d, dtype=np.float64)
    shape = d.shape[:-1]
    d = d.reshape(-1, 3)
    R = np.sqrt(np.sum(d * d, axis=-1))
    kr = k * R
    g = scalar_g(R, k)
    A = 1.0 - 1j / kr - 1.0 / kr ** 2
    B = -1.0 + 3j / kr + 3.0 / kr ** 2
    dh = d / R[:, None]
    G = g[:, None, None] * (A[:, None, None] * np.eye(3)
                            + B[:, None, None] * dh[:, :, None] * dh[:, None, :])
    return G.reshape(shape + (3, 3))


def self_term(a: np.ndarray | float, k: float):
    """s(a): k^2 PV-integral of G over the equal-volume sphere, plus -1/3."""
    ka = k * np.asarray(a, dtype=np.float64)
    return (2.0 / 3.0) * ((1.0 + 1j * ka) * np.exp(-1j * ka) - 1.0) - 1.0 / 3.0


def _pair_block(pos_r, vol_r, pos_c, vol_c, k):
    """Off-diagonal entries for all (row cell, col cell) pairs, (nr*3, nc*3)."""
    d = pos_r[:, None, :] - pos_c[None, :, :]
    G = dyadic(d, k)                                  # (nr, nc, 3, 3)
    Z = (-k * k) * (vol_r[:, None] * vol_c[None, :])[:, :, None, None] * G
    nr, nc = pos_r.shape[0], pos_c.shape[0]
    return Z.transpose(0, 2, 1, 3).reshape(nr * 3, nc * 3)


def particle_self_block(disc, p: int) -> np.ndarray:
    """Z_pp (144 x 144) of particle p, built from the cell offsets."""
    off = disc.offsets[p]
    v = np.full(N_CELLS, disc.vol[p])
    d = off[:, None, :] - off[None, :, :]
    idx = np.arange(N_CELLS)
    d[idx, idx, 0] = 1.0                              # placeholder on the diagonal
    G = dyadic(d, disc.k)
    Z = (-disc.k ** 2) * (v[:, None] * v[None, :])[:, :, None, None] * G
    diag = disc.vol[p] * (1.0 / disc.chi[p] - self_term(disc.a_eq[p], disc.k))
    Z[idx, idx] = diag * np.eye(3)
    return Z.transpose(0, 2, 1, 3).reshape(N_DOF_PER_PARTICLE, N_DOF_PER_PARTICLE)


def assemble_block(disc, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """Z restricted to particles `rows` x `cols` (caller particle indices).

    Row/column DoFs follow the order of the given particle lists.  Self blocks
    (p, p) are taken from ``particle_self_block``.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    out = np.empty((rows.size * N_DOF_PER_PARTICLE, cols.size * N_DOF_PER_PARTICLE),
                   dtype=np.complex128)
    for bi, p in enumerate(rows):
        rsl = slice(bi * N_DOF_PER_PARTICLE, (bi + 1) * N_DOF_PER_PARTICLE)
        # all distinct columns at once
        distinct = cols != p
        if np.any(distinct):
            cq = cols[distinct]
            pos_c = disc.pos[cq].reshape(-1, 3)
            vol_c = np.repeat(disc.vol[cq], N_CELLS)
            blk = _pair_block(disc.pos[p], np.full(N_CELLS, disc.vol[p]), pos_c, vol_c, disc.k)
            colidx = np.nonzero(distinct)[0]
            for t, bj in enumerate(colidx):
                out[rsl, bj * N_DOF_PER_PARTICLE:(bj + 1) * N_DOF_PER_PARTICLE] = \
                    blk[:, t * N_DOF_PER_PARTICLE:(t + 1) * N_DOF_PER_PARTICLE]
        for bj in np.nonzero(~distinct)[0]:
            out[rsl, bj * N_DOF_PER_PARTICLE:(bj + 1) * N_DOF_PER_PARTICLE] = \
                particle_self_block(disc, p)
    return out


def assemble_dense(disc) -> np.ndarray:
    """Full Z (ndof x ndof), particle-major caller order."""
    allp = np.arange(disc.n_particles)
    return assemble_block(disc, allp, allp)


def matvec_free(disc, x: np.ndarray, rows: np.ndarray | None = None,
                chunk: int = 8) -> np.ndarray:
    """y = Z x without storing Z; optionally only for particle rows `rows`.

    x is (ndof,) or (ndof, nrhs).  Entries are regenerated chunk by chunk.
    """
    x2 = x.reshape(x.shape[0], -1)
    allp = np.arange(disc.n_particles)
    rows = allp if rows is None else np.asarray(rows)
    y = np.zeros((rows.size * N_DOF_PER_PARTICLE, x2.shape[1]), dtype=np.complex128)
    for s in range(0, rows.size, chunk):
        rr = rows[s:s + chunk]
        blk = assemble_block(disc, rr, allp)
        y[s * N_DOF_PER_PARTICLE:(s + rr.size) * N_DOF_PER_PARTICLE] = blk @ x2
    return y.reshape((-1,) + x.shape[1:])


def plane_wave_rhs(disc, theta_deg, phi_deg, pol) -> np.ndarray:
    """v0 for plane waves (ndof, nrhs); pol 0 = TE, 1 = TM.

    k^ = (sin t cos f, sin t sin f, cos t); TE e = (-sin f, cos f, 0);
    TM e = (cos t cos f, cos t sin f, -sin t).
    """
    theta = np.deg2rad(np.atleast_1d(theta_deg).astype(np.float64))
    phi = np.deg2rad(np.atleast_1d(phi_deg).astype(np.float64))
    pol = np.atleast_1d(pol)
    pos, vol, _, _ = disc.cell_arrays()
    out = np.zeros((pos.shape[0] * 3, theta.size), dtype=np.complex128)
    for r in range(theta.size):
        t, f = theta[r], phi[r]
        khat = np.array([math.sin(t) * math.cos(f), math.sin(t) * math.sin(f), math.cos(t)])
        if pol[r] == 0:
            e = np.array([-math.sin(f), math.cos(f), 0.0])
        else:
            e = np.array([math.cos(t) * math.cos(f), math.cos(t) * math.sin(f), -math.sin(t)])
        phase = np.exp(-1j * disc.k * (pos @ khat))
        out[:, r] = (vol[:, None] * phase[:, None] * e[None, :]).reshape(-1)
    return out


def self_blocks(disc) -> np.ndarray:
    """(N, 144, 144) diagonal blocks Z_pp (the near part left at the finest level, §5.4)."""
    return np.stack([particle_self_block(disc, p) for p in range(disc.n_particles)])
