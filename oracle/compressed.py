"""Checks of low-rank factors and the compressed product (oracle, FP64).

The method replaces each far block B (m x n) by Q (m x r) R (r x n) within a
prescribed tolerance (§5.2, eq. 5.3) and applies it as Q (R x).  The reading of
"within tolerance eps" used throughout is per block, relative Frobenius:
||B - Q R||_F <= eps ||B||_F.  Because blocks have disjoint supports this
implies ||(Z_QR - Z) x|| <= eps ||Z_off||_F ||x|| for the whole operator.

This module takes factors as *data* (exported by the GPU library, or produced
in tests by ``qrcp_truncate``) and checks them against its own re-assembly:

* ``check_block``: relative error, orthonormality of Q, and the Eckart-Young
  lower bound on the rank (smallest r whose SVD tail is <= eps ||B||_F);
* ``compressed_apply``: y = Z_D x + sum_b Q_b (R_b x_J), the product of §5.2;
* ``eps_prod``: the accuracy metric of §6.2 with u = (1 + j) [1 ... 1]^T;
* ``gain``: G = N_dof^2 / N_QR of §5.3, eq. 5.5-5.6.

``qrcp_truncate`` is the oracle's own low-rank QR (column-pivoted Householder QR
through scipy, truncated at the smallest rank meeting the tolerance); it is the
reference the GPU's ranks and solution accuracy are compared with.

Pins (tests): ``svd_rank`` on blocks with prescribed singular values, at and around
every tail threshold, and as the Eckart-Young minimum of the truncated SVD;
``dense_from_factors`` against blocks placed by hand particle by particle;
``compressed_apply`` equals that dense operator; ``eps_prod`` and ``gain`` against
hand-computed cases; per-block eps met with orthonormal Q and ranks at or above the SVD
bound; the global product bound ||(Z_QR - Z) x|| <= eps ||Z_off||_F ||x||; eps_prod < eps;
tighter eps lowers G and raises the solution accuracy (the trends of §6.2).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .discretise import N_DOF_PER_PARTICLE


def svd_rank(B: np.ndarray, eps: float) -> int:
    s = np.linalg.svd(B, compute_uv=False)
    tot = np.sum(s ** 2)
    tail = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]])
    r = int(np.argmax(tail <= eps * eps * tot))
    return r


def qrcp_truncate(B: np.ndarray, eps: float):
    """Q (m x r), R (r x n) from pivoted QR, r minimal with trailing norm <= eps ||B||_F."""
    Q, R, P = scipy.linalg.qr(B, mode="economic", pivoting=True)
    tot = np.linalg.norm(B) ** 2
    rownorm2 = np.sum(np.abs(R) ** 2, axis=1)
    tail = np.concatenate([np.cumsum(rownorm2[::-1])[::-1], [0.0]])
    r = int(np.argmax(tail <= eps * eps * tot))
    Rr = np.zeros((r, B.shape[1]), dtype=np.complex128)
    Rr[:, P] = R[:r, :]
    return Q[:, :r], Rr


def check_block(B: np.ndarray, Q: np.ndarray, R: np.ndarray, eps: float) -> dict:
    nb = np.linalg.norm(B)
    err = np.linalg.norm(B - Q @ R) / nb if nb > 0 else 0.0
    r = Q.shape[1]
    ortho = np.max(np.abs(Q.conj().T @ Q - np.eye(r))) if r else 0.0
    return dict(rel_err=float(err), ortho=float(ortho), rank=r,
                svd_rank=svd_rank(B, eps), ok=bool(err <= eps))


def particle_dofs(particles) -> np.ndarray:
    """DoF indices (caller order) of a list of particles."""
    p = np.asarray(particles, dtype=np.int64)
    return (p[:, None] * N_DOF_PER_PARTICLE + np.arange(N_DOF_PER_PARTICLE)[None, :]).reshape(-1)


def factor_apply(factors, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """y += sum over blocks of Q (R x_J): the far part of the product, in the order of §5.2."""
    for rows, cols, Q, R in factors:
        ri = particle_dofs(rows)
        ci = particle_dofs(cols)
        y[ri] += Q @ (R @ x[ci])
    return y


def compressed_apply(self_blocks: np.ndarray, factors, x: np.ndarray) -> np.ndarray:
    """Z_QR x = Z_D x + sum over blocks of Q (R x_J).

    factors: iterable of (row particles, col particles, Q, R).
    """
    n = self_blocks.shape[0]
    nb = self_blocks.shape[1]
    x2 = x.reshape(n * nb, -1)
    y = np.einsum("pij,pjk->pik", self_blocks, x2.reshape(n, nb, -1)).reshape(n * nb, -1)
    factor_apply(factors, x2, y)
    return y.reshape(x.shape)


def dense_from_factors(self_blocks: np.ndarray, factors) -> np.ndarray:
    n, nb = self_blocks.shape[0], self_blocks.shape[1]
    Z = np.zeros((n * nb, n * nb), dtype=np.complex128)
    for p in range(n):
        Z[p * nb:(p + 1) * nb, p * nb:(p + 1) * nb] = self_blocks[p]
    for rows, cols, Q, R in factors:
        ri = particle_dofs(rows)
        ci = particle_dofs(cols)
        Z[np.ix_(ri, ci)] += Q @ R
    return Z


def eps_prod(apply_qr, apply_dense, ndof: int) -> float:
    u = (1.0 + 1.0j) * np.ones(ndof)
    zu = apply_dense(u)
    return float(np.linalg.norm(apply_qr(u) - zu) / np.linalg.norm(zu))


def gain(ndof: int, n_self_entries: int, factors_ranks) -> float:
    """G = N_dof^2 / N_QR with N_QR = sum (m + n) r + N N_p^2 (eqs. 5.5-5.6)."""
    nqr = n_self_entries + sum((m + n) * r for m, n, r in factors_ranks)
    return ndof * ndof / nqr
