"""Pins of the oracle's factor checkers and of GMRES's intermediate iterates (no GPU).

The GPU tests lean on four oracle functions beyond the physics: the Eckart-Young rank
bound ``svd_rank``, the dense assembly of a factored operator ``dense_from_factors``,
the compressed product ``compressed_apply`` and the product accuracy ``eps_prod`` of
§6.2.  Each is pinned here by values fixed by construction (prescribed singular values,
hand-placed entries, a hand-computed perturbation), chosen so that an off-by-one in a
tail sum, a transposed or misplaced block, or a wrong probe vector fails.  GMRES(m)
stopped after m steps is pinned to the least-squares minimiser over the Krylov space,
built here from explicit matrix powers (the definition, not the Arnoldi recurrence).
"""
import numpy as np
import pytest

from oracle import compressed, solvers


def _unitary(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _with_singular_values(s, m, n, seed):
    rng = np.random.default_rng(seed)
    U, V = _unitary(rng, m)[:, :len(s)], _unitary(rng, n)[:, :len(s)]
    return (U * np.asarray(s)) @ V.conj().T


# singular values 1, 1e-2, 1e-4, 1e-6, 1e-8.  ||B||_F = sqrt(1.0001000100010001) and the
# tails after r values are, relative to ||B||_F:
#   r = 0: 1;  r = 1: 1.00005e-2 / 1.00005 = 1.0000e-2 (to 5 digits);  r = 2: 1.0000e-4;
#   r = 3: 1.0000e-6;  r = 4: 1e-8 / 1.00005 = 0.99995e-8;  r = 5: 0.
SV = [1.0, 1e-2, 1e-4, 1e-6, 1e-8]


@pytest.mark.parametrize("eps,rank", [
    (2.0, 0), (0.9999, 1), (1.01e-2, 1), (0.99e-2, 2), (1.01e-4, 2), (0.99e-4, 3),
    (1.01e-6, 3), (0.99e-6, 4), (1.01e-8, 4), (0.98e-8, 5), (1e-12, 5),
])
def test_svd_rank_on_prescribed_singular_values(eps, rank):
    B = _with_singular_values(SV, 40, 30, seed=1)
    assert compressed.svd_rank(B, eps) == rank


def test_svd_rank_of_a_zero_block_is_zero():
    assert compressed.svd_rank(np.zeros((6, 4), complex), 1e-6) == 0


def test_svd_rank_is_the_eckart_young_minimum():
    """Truncating the SVD at svd_rank meets eps; one fewer singular value does not."""
    s = np.exp(-0.7 * np.arange(25))
    B = _with_singular_values(s, 50, 35, seed=4)
    for eps in (1e-2, 1e-4, 1e-6):
        r = compressed.svd_rank(B, eps)
        U, sv, Vh = np.linalg.svd(B, full_matrices=False)
        err = lambda k: np.linalg.norm(B - (U[:, :k] * sv[:k]) @ Vh[:k]) / np.linalg.norm(B)
        assert err(r) <= eps < err(r - 1)
        assert isinstance(r, int)


def _random_factors(rng, nparticles, nb=144):
    """A few blocks on particle lists of different lengths, in scrambled particle order."""
    blocks = []
    for rows, cols, r in (([2, 0], [1], 3), ([1], [3, 2], 2), ([3], [0, 2], 4), ([0, 1], [3], 1)):
        Q = rng.standard_normal((len(rows) * nb, r)) + 1j * rng.standard_normal((len(rows) * nb, r))
        R = rng.standard_normal((r, len(cols) * nb)) + 1j * rng.standard_normal((r, len(cols) * nb))
        blocks.append((rows, cols, Q, R))
    sb = rng.standard_normal((nparticles, nb, nb)) + 1j * rng.standard_normal((nparticles, nb, nb))
    return sb, blocks


def test_dense_from_factors_places_every_block_by_hand():
    """Particle block (p, q) of the assembled operator is Z_pp on the diagonal plus block
    (i, j) of Q R for every factored block whose i-th row particle is p and j-th column
    particle is q, placed here with explicit loops over the particle lists."""
    rng = np.random.default_rng(6)
    sb, blocks = _random_factors(rng, 4)
    Z = compressed.dense_from_factors(sb, blocks)
    nb = 144
    ref = np.zeros((4 * nb, 4 * nb), complex)
    for p in range(4):
        ref[p * nb:(p + 1) * nb, p * nb:(p + 1) * nb] += sb[p]
    for rows, cols, Q, R in blocks:
        P = Q @ R
        for i, p in enumerate(rows):
            for j, q in enumerate(cols):
                ref[p * nb:(p + 1) * nb, q * nb:(q + 1) * nb] += P[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
    assert np.array_equal(Z, ref)


def test_compressed_apply_equals_the_dense_operator():
    rng = np.random.default_rng(7)
    sb, blocks = _random_factors(rng, 4)
    Z = compressed.dense_from_factors(sb, blocks)
    x = rng.standard_normal((4 * 144, 3)) + 1j * rng.standard_normal((4 * 144, 3))
    y = compressed.compressed_apply(sb, blocks, x)
    assert np.linalg.norm(y - Z @ x) <= 1e-13 * np.linalg.norm(Z @ x)
    y1 = compressed.compressed_apply(sb, blocks, x[:, 1])
    assert np.linalg.norm(y1 - Z @ x[:, 1]) <= 1e-13 * np.linalg.norm(Z @ x[:, 1])


def test_eps_prod_by_hand():
    """Dense operator 2 I; compressed operator 2 I plus d Im(u_0) in entry 0.  With the
    probe u = (1 + j)[1 ... 1] of §6.2, ||(Z_QR - Z) u|| = d and ||Z u|| = 2 sqrt(2 n), so
    eps_prod = d / (2 sqrt(2 n)).  A probe without the imaginary unit gives 0 instead."""
    n, d = 50, 3e-7

    def dense(u):
        return 2.0 * u

    def qr(u):
        y = 2.0 * u
        y[0] += d * u[0].imag
        return y

    assert compressed.eps_prod(qr, dense, n) == pytest.approx(d / (2 * np.sqrt(2 * n)), rel=1e-12)


def test_gain_by_hand():
    """Two blocks (m, n, r) = (288, 144, 10), (144, 288, 4): N_QR = 2 * 144^2 + 4320 + 1728."""
    g = compressed.gain(288, 2 * 144 * 144, [(288, 144, 10), (144, 288, 4)])
    assert g == pytest.approx(288 * 288 / (2 * 144 * 144 + 4320 + 1728), rel=1e-15)


def _krylov_minimiser(A, M, b, m):
    """argmin ||M (b - A x)|| over x in span{c, (MA) c, ..., (MA)^{m-1} c}, c = M b,
    from explicit powers orthonormalised by QR (the definition of the m-th GMRES iterate)."""
    MA = M @ A
    K = np.empty((b.size, m), complex)
    K[:, 0] = M @ b
    for j in range(1, m):
        K[:, j] = MA @ K[:, j - 1]
        K[:, j] /= np.linalg.norm(K[:, j])
    Qk, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(MA @ Qk, M @ b, rcond=None)
    return Qk @ y


@pytest.mark.parametrize("m", [3, 6, 10])
def test_gmres_after_m_steps_is_the_krylov_minimiser(m):
    """GMRES(m) stopped after exactly m steps (x0 = 0) returns the minimiser of the
    preconditioned residual over the m-dimensional Krylov space, and reports that
    residual explicitly.  A well-conditioned system keeps the power basis usable."""
    rng = np.random.default_rng(m)
    n = 40
    A = np.eye(n) * 4 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    Mi = np.eye(n) + 0.1 * np.diag(rng.standard_normal(n))
    M = np.linalg.inv(Mi)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = solvers.gmres(lambda v: A @ v, b, apply_M=lambda v: M @ v, restart=m, tol=1e-15, max_iter=m)
    ref = _krylov_minimiser(A, M, b, m)
    assert info.iterations == m and not info.converged
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    explicit = np.linalg.norm(M @ (b - A @ x)) / np.linalg.norm(M @ b)
    assert info.rel_res_prec == pytest.approx(explicit, rel=1e-12)
    assert info.history[-1] == pytest.approx(explicit, rel=1e-6)
