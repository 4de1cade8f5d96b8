"""Pins of the oracle's direct and iterative solvers (no GPU)."""
import numpy as np
import pytest

import workloads as W
from oracle import compressed, discretise, greens, grouping, solvers


def test_own_lu_matches_lapack():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((60, 60)) + 1j * rng.standard_normal((60, 60))
    b = rng.standard_normal(60) + 1j * rng.standard_normal(60)
    x = solvers.lu_solve(solvers.lu_factor(A), b)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) / np.linalg.norm(x) < 1e-12


def test_block_preconditioner_is_exact_inverse_of_block_diagonal(tiny_oracle):
    sb = tiny_oracle["self_blocks"]
    P = solvers.BlockDiagPreconditioner(sb)
    assert P.n_distinct == 1            # identical atoms: one factorisation (§4)
    x = np.random.default_rng(2).standard_normal(sb.shape[0] * 144) + 0j
    y = np.einsum("pij,pj->pi", sb, x.reshape(16, 144)).reshape(-1)
    assert np.linalg.norm(P.apply(y) - x) / np.linalg.norm(x) < 1e-12


def test_gmres_matches_lu_on_tiny(tiny_oracle):
    Z, v, xlu = tiny_oracle["Z"], tiny_oracle["v"], tiny_oracle["x_lu"]
    P = solvers.BlockDiagPreconditioner(tiny_oracle["self_blocks"])
    x, info = solvers.gmres(lambda u: Z @ u, v, P.apply, restart=30, tol=1e-10)
    assert info.converged
    assert np.linalg.norm(x - xlu) / np.linalg.norm(xlu) < 1e-7
    # residual estimates are monotone within a cycle
    h = np.array(info.history[:30])
    assert np.all(np.diff(h) <= 1e-14)


def test_givens_estimate_equals_the_explicit_preconditioned_residual(tiny_oracle):
    """After one cycle of m steps, the rotated right-hand side |g_(m+1)| / ||M b|| is the
    preconditioned residual of the iterate the cycle returns (a GMRES identity)."""
    Z, v = tiny_oracle["Z"], tiny_oracle["v"]
    P = solvers.BlockDiagPreconditioner(tiny_oracle["self_blocks"])
    mb = np.linalg.norm(P.apply(v))
    for m in (1, 5, 10, 17):
        x, info = solvers.gmres(lambda u: Z @ u, v, P.apply, restart=m, tol=1e-14, max_iter=m)
        explicit = np.linalg.norm(P.apply(v - Z @ x)) / mb
        assert len(info.history) == m
        assert abs(info.history[-1] - explicit) <= 1e-8 * explicit


def test_single_particle_converges_in_one_iteration():
    """The preconditioner is the exact inverse for an isolated meta-atom (§4)."""
    arr = W.lattice(1, radius=0.2)
    d = discretise.Discretisation(arr)
    Z = greens.assemble_dense(d)
    v = greens.plane_wave_rhs(d, [0.0], [0.0], [1])[:, 0]
    P = solvers.BlockDiagPreconditioner(greens.self_blocks(d))
    x, info = solvers.gmres(lambda u: Z @ u, v, P.apply, restart=10, tol=1e-12)
    assert info.converged and info.iterations == 1


def test_preconditioner_cuts_iterations_by_orders_of_magnitude(tiny_oracle):
    """Qualitative pin of the paper's 53 vs 9067 iterations (§6.3)."""
    Z, v = tiny_oracle["Z"], tiny_oracle["v"]
    P = solvers.BlockDiagPreconditioner(tiny_oracle["self_blocks"])
    _, with_p = solvers.gmres(lambda u: Z @ u, v, P.apply, restart=30, tol=1e-6)
    _, without = solvers.gmres(lambda u: Z @ u, v, None, restart=30, tol=1e-6, max_iter=600)
    assert with_p.converged and with_p.iterations < 40
    assert not without.converged          # stagnates far beyond 15x the preconditioned count


def test_weak_coupling_needs_few_iterations():
    """Pitch -> large: mutual interactions vanish and Z_D^-1 becomes exact."""
    iters = []
    for pitch in (0.5, 4.0, 64.0):
        arr = W.lattice(2, 2, pitch=pitch, radius=0.2)
        d = discretise.Discretisation(arr)
        Z = greens.assemble_dense(d)
        v = greens.plane_wave_rhs(d, [0.0], [0.0], [1])[:, 0]
        P = solvers.BlockDiagPreconditioner(greens.self_blocks(d))
        _, info = solvers.gmres(lambda u: Z @ u, v, P.apply, restart=50, tol=1e-10)
        iters.append(info.iterations)
    assert iters[0] > iters[1] > iters[2]


def test_compressed_operator_accuracy_bounds(tiny_oracle):
    """Per-block eps (eq. 5.3 reading) implies the global product bound; eps trends (§6.2)."""
    d, Z, v, xlu = tiny_oracle["disc"], tiny_oracle["Z"], tiny_oracle["v"], tiny_oracle["x_lu"]
    sb = tiny_oracle["self_blocks"]
    arr = tiny_oracle["array"]
    blocks = grouping.build_blocks(arr.lattice_ij, 4, 4)
    Zoff = Z.copy()
    for p in range(16):
        Zoff[p * 144:(p + 1) * 144, p * 144:(p + 1) * 144] = 0
    x = np.random.default_rng(5).standard_normal(Z.shape[0]) * (1 + 0.5j)
    gains, errs = [], []
    for eps in (1e-3, 1e-6):
        fac, ranks = [], []
        for b in blocks:
            B = greens.assemble_block(d, b.rows, b.cols)
            Q, R = compressed.qrcp_truncate(B, eps)
            chk = compressed.check_block(B, Q, R, eps)
            assert chk["ok"] and chk["ortho"] < 1e-12 and chk["rank"] >= chk["svd_rank"]
            fac.append((b.rows, b.cols, Q, R))
            ranks.append((B.shape[0], B.shape[1], Q.shape[1]))
        y = compressed.compressed_apply(sb, fac, x)
        assert np.linalg.norm(y - Z @ x) <= eps * np.linalg.norm(Zoff) * np.linalg.norm(x)
        ep = compressed.eps_prod(lambda u: compressed.compressed_apply(sb, fac, u),
                                 lambda u: Z @ u, Z.shape[0])
        assert ep < eps
        ZQR = compressed.dense_from_factors(sb, fac)
        errs.append(np.linalg.norm(np.linalg.solve(ZQR, v) - xlu) / np.linalg.norm(xlu))
        gains.append(compressed.gain(Z.shape[0], 16 * 144 * 144, ranks))
        # N_QR is the number of complex entries actually stored: self blocks plus Q and R
        stored = sb.size + sum(Q.size + R.size for _, _, Q, R in fac)
        assert gains[-1] == pytest.approx(Z.shape[0] ** 2 / stored, rel=1e-15)
        assert ZQR.shape == Z.shape and stored < Z.size
    # tighter eps: lower gain, higher solution accuracy (the trend of §6.2)
    assert gains[0] > gains[1] > 1.0
    assert errs[0] > errs[1]
