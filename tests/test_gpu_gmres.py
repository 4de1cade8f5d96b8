"""GMRES intermediate state on the GPU against the oracle (§6 solver with the left
preconditioner of §4).

GMRES(m) stopped after exactly m Arnoldi steps from x0 = 0 returns the minimiser of the
preconditioned residual over the m-dimensional Krylov space, a unique vector whatever
orthogonalisation builds the basis.  The library (classical Gram-Schmidt whose second
projection goes through the basis Gram matrix) and the oracle (modified Gram-Schmidt, pinned
to the least-squares definition on the CPU) must therefore return the same x_m, and the
library's reported preconditioned residual must equal the oracle's explicit
||Z_D^-1 (v - Z_QR x_m)|| / ||Z_D^-1 v||.  This pins the Arnoldi and Givens state before
convergence, not only converged solutions; the loss of orthogonality of the stored basis is
read from the library's own Gram matrix.
"""
import numpy as np
import pytest

from oracle import compressed, greens, solvers

from gpu_cases import case, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m", [5, 20, 40])
def test_gmres_iterate_after_m_steps_matches_the_oracle(m):
    import paper_2603_10586_amd as q
    c = case("rand6x7")
    v = q.rhs_plane_waves(c.ctx, c.geom, [10.0], [0.0], [1])
    x, info, st = c.op.solve(v, restart=m, tol=1e-15, max_iter=m)
    assert st == 5 and info[0]["iterations"] == m and info[0]["restarts"] == 1
    sb = greens.self_blocks(c.disc)
    ZQR = compressed.dense_from_factors(sb, [(f[0], f[1], f[2], f[3]) for f in c.factors()])
    P = solvers.BlockDiagPreconditioner(sb)
    vh = to_host(v)[0]
    xo, io = solvers.gmres(lambda u: ZQR @ u, vh, apply_M=P.apply, restart=m, tol=1e-15, max_iter=m)
    assert io.iterations == m
    xh = to_host(x)[0]
    assert np.linalg.norm(xh - xo) <= 1e-8 * np.linalg.norm(xo)
    explicit = np.linalg.norm(P.apply(vh - ZQR @ xh)) / np.linalg.norm(P.apply(vh))
    assert info[0]["rel_res_prec"] == pytest.approx(explicit, rel=1e-6)
    assert info[0]["rel_res_prec"] == pytest.approx(io.rel_res_prec, rel=1e-5)
    assert info[0]["rel_res_true"] == pytest.approx(np.linalg.norm(vh - ZQR @ xh) / np.linalg.norm(vh), rel=1e-6)
    assert 0.0 < info[0]["basis_ortho"] <= 1e-12


def test_gmres_residuals_decrease_with_the_krylov_dimension():
    """The minimiser over a larger Krylov space has a smaller preconditioned residual."""
    import paper_2603_10586_amd as q
    c = case("rand6x7")
    v = q.rhs_plane_waves(c.ctx, c.geom, [0.0], [0.0], [0])
    res = []
    for m in (4, 8, 16, 32):
        _, info, _ = c.op.solve(v, restart=m, tol=1e-15, max_iter=m)
        res.append(info[0]["rel_res_prec"])
    assert all(b < a for a, b in zip(res, res[1:])), res
