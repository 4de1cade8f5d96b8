"""Direct and iterative solvers of Z I = v0 (oracle, FP64).

* ``lu_factor`` / ``lu_solve``: Gaussian elimination with partial pivoting
  written out (the paper's direct reference solution, §6.2, A_s metric);
  ``numpy.linalg.solve`` is the library cross-check.
* ``BlockDiagPreconditioner``: the left preconditioner Z_D^-1, the exact
  inverse of the particle block diagonal (§4, eqs. 4.1-4.2), one LU per
  distinct self block.
* ``gmres``: left-preconditioned restarted GMRES (the paper's solver, §6) with
  modified Gram-Schmidt Arnoldi and complex Givens rotations on the
  Hessenberg matrix.  x0 = 0.  The iteration works on the preconditioned
  residual; a solve counts as converged only when the explicit true residual
  ||v - Z x|| / ||v|| also meets the tolerance (otherwise it restarts).

Pins (tests): own LU == numpy.linalg.solve; GMRES == LU on small systems;
one particle converges in one iteration (preconditioner exact for an isolated
meta-atom, §4); after one cycle the Givens estimate equals the explicit preconditioned
residual of the returned iterate; estimates are monotone within a cycle; GMRES(m)
stopped after m steps equals the least-squares minimiser over the Krylov space built
from explicit matrix powers.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def lu_factor(A: np.ndarray):
    """PA = LU with partial pivoting; returns (LU packed, piv)."""
    A = np.array(A, dtype=np.complex128, copy=True)
    n = A.shape[0]
    piv = np.arange(n)
    for k in range(n):
        p = k + int(np.argmax(np.abs(A[k:, k])))
        if p != k:
            A[[k, p]] = A[[p, k]]
            piv[[k, p]] = piv[[p, k]]
        if A[k, k] == 0:
            raise np.linalg.LinAlgError("singular matrix")
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return A, piv


def lu_solve(fac, b: np.ndarray) -> np.ndarray:
    LU, piv = fac
    n = LU.shape[0]
    y = np.array(b, dtype=np.complex128)[piv]
    for i in range(n):                       # forward, unit lower
        y[i] -= LU[i, :i] @ y[:i]
    for i in range(n - 1, -1, -1):           # backward, upper
        y[i] = (y[i] - LU[i, i + 1:] @ y[i + 1:]) / LU[i, i]
    return y


class BlockDiagPreconditioner:
    """z = Z_D^-1 y, with Z_D = diag(Z_11, ..., Z_NN) (§4, eq. 4.2)."""

    def __init__(self, self_blocks: np.ndarray):
        self.nb = self_blocks.shape[1]
        self.n = self_blocks.shape[0]
        # identical blocks share one factorisation (§4: O(1) for identical atoms)
        self._inv = []
        cache = {}
        for p in range(self.n):
            key = self_blocks[p].tobytes()
            if key not in cache:
                cache[key] = np.linalg.inv(self_blocks[p])
            self._inv.append(cache[key])
        self.n_distinct = len(cache)

    def apply(self, y: np.ndarray) -> np.ndarray:
        y2 = y.reshape(self.n, self.nb, -1)
        z = np.empty_like(y2, dtype=np.complex128)
        for p in range(self.n):
            z[p] = self._inv[p] @ y2[p]
        return z.reshape(y.shape)


@dataclass
class GmresInfo:
    iterations: int = 0
    restarts: int = 0
    converged: bool = False
    rel_res_prec: float = np.inf
    rel_res_true: float = np.inf
    history: list = field(default_factory=list)


def _givens(a: complex, b: complex):
    """(c, s) with c real so that [[c, s], [-conj(s), c]] @ [a, b] = [rho, 0]."""
    if b == 0:
        return 1.0, 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    rho = np.hypot(abs(a), abs(b))
    c = abs(a) / rho
    s = (a / abs(a)) * np.conj(b) / rho
    return c, s


def gmres(apply_A, b: np.ndarray, apply_M=None, restart: int = 30, tol: float = 1e-8,
          max_iter: int = 10000, x0: np.ndarray | None = None) -> tuple[np.ndarray, GmresInfo]:
    """Left-preconditioned GMRES(restart): solves M A x = M b.

    Stops when the preconditioned residual estimate <= tol * ||M b|| and the
    true residual ||b - A x|| <= tol * ||b||.
    """
    M = apply_M if apply_M is not None else (lambda v: v)
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    info = GmresInfo()
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        info.converged, info.rel_res_prec, info.rel_res_true = True, 0.0, 0.0
        return x, info
    mb_norm = np.linalg.norm(M(b))
    prec_tol = tol
    while info.iterations < max_iter:
        r = M(b - apply_A(x))
        beta = np.linalg.norm(r)
        info.rel_res_prec = beta / mb_norm
        if info.rel_res_prec <= prec_tol:
            true_rel = np.linalg.norm(b - apply_A(x)) / bnorm
            info.rel_res_true = true_rel
            if true_rel <= tol:
                info.converged = True
                return x, info
            prec_tol = prec_tol * 0.5 * tol / max(true_rel, 1e-300)
        m = restart
        V = np.zeros((n, m + 1), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[:, 0] = r / beta
        k_used = 0
        for j in range(m):
            w = M(apply_A(V[:, j]))
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            for i in range(j):                           # previous rotations
                a, bb = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * bb
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * bb
            c, s = _givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j] = c * H[j, j] + s * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            info.iterations += 1
            k_used = j + 1
            est = abs(g[j + 1]) / mb_norm
            info.history.append(est)
            if hn != 0:
                V[:, j + 1] = w / hn
            if est <= prec_tol or hn == 0 or info.iterations >= max_iter:
                break
        y = np.zeros(k_used, dtype=np.complex128)
        for i in range(k_used - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k_used] @ y[i + 1:k_used]) / H[i, i]
        x = x + V[:, :k_used] @ y
        info.restarts += 1
    r = M(b - apply_A(x))
    info.rel_res_prec = np.linalg.norm(r) / mb_norm
    info.rel_res_true = np.linalg.norm(b - apply_A(x)) / bnorm
    info.converged = info.rel_res_prec <= tol and info.rel_res_true <= tol
    return x, info
