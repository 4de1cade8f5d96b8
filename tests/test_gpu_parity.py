"""GPU path vs the FP64 oracle on small arrays, through the C ABI.

Tolerances: entries of Z and v0 are evaluated by both sides from the same formulas
in FP64 with different libm implementations and operation orders, so they agree to
a few ulps of the largest entry (1e-13 relative is asserted).  Products of the same
operator agree to accumulated rounding (1e-12).  Low-rank factors are not unique
(§5.2 only fixes the tolerance), so blocks are checked by the certified error
||B - QR||_F <= eps ||B||_F against the oracle's own B, and products/solutions are
compared instead of factors.  Solutions: same-operator parity 1e-6 (north-star
field tolerance), method accuracy against the uncompressed LU within 3x the
oracle's own QRCP compression at the same eps.
"""
import numpy as np
import pytest

import workloads as W
from oracle import compressed, greens, solvers

from gpu_cases import case, to_dev, to_host

pytestmark = pytest.mark.gpu

NAMES = ["tiny", "rand5x3", "rand6x7"]


@pytest.mark.parametrize("name", NAMES)
def test_cells_match_oracle(name):
    c = case(name)
    centers, vols = c.geom.cells()
    pos, vol, _, _ = c.disc.cell_arrays()
    assert np.max(np.abs(centers - pos)) <= 1e-15
    assert np.max(np.abs(vols - vol) / vol) <= 1e-15


@pytest.mark.parametrize("name", NAMES)
def test_assembly_matches_oracle(name):
    import paper_2603_10586_amd as q
    c = case(name)
    n = c.array.n_particles
    rng = np.random.default_rng(0)
    rows = rng.choice(n, size=min(3, n), replace=False)
    cols = np.concatenate([rows[:1], rng.choice(n, size=min(4, n), replace=False)])
    B = to_host(q.assemble(c.ctx, c.geom, rows, cols))
    ref = greens.assemble_block(c.disc, rows, cols)
    assert B.shape == ref.shape
    assert np.max(np.abs(B - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("name", NAMES)
def test_plane_wave_rhs_matches_oracle(name):
    import paper_2603_10586_amd as q
    c = case(name)
    th, ph, po = [0.0, 10.0, -27.5], [0.0, 0.0, 33.0], [1, 1, 0]
    v = to_host(q.rhs_plane_waves(c.ctx, c.geom, th, ph, po)).T
    ref = greens.plane_wave_rhs(c.disc, th, ph, po)
    assert np.max(np.abs(v - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("name", NAMES)
def test_self_blocks_and_preconditioner_inverse(name):
    c = case(name)
    for p in range(0, c.array.n_particles, max(1, c.array.n_particles // 5)):
        Z, Zi = c.op.export_self(p)
        ref = greens.particle_self_block(c.disc, p)
        assert np.max(np.abs(Z - ref)) <= 1e-13 * np.max(np.abs(ref))
        assert np.max(np.abs(Zi @ ref - np.eye(144))) <= 1e-11


@pytest.mark.parametrize("name", NAMES)
def test_block_list_matches_oracle_grouping(name):
    c = case(name)
    gpu = sorted((f[4]["level"], tuple(sorted(f[0])), tuple(sorted(f[1]))) for f in c.factors())
    ora = sorted((b.level, tuple(sorted(b.rows)), tuple(sorted(b.cols))) for b in c.oracle_blocks())
    assert gpu == ora


@pytest.mark.parametrize("name", NAMES)
def test_every_block_is_certified_against_the_oracle(name):
    c = case(name)
    mirror_checked = 0
    by_key = {(tuple(f[0]), tuple(f[1])): f for f in c.factors()}
    for rows, cols, Q, R, info in c.factors():
        B = greens.assemble_block(c.disc, rows, cols)
        err = np.linalg.norm(B - Q @ R) / np.linalg.norm(B)
        assert err <= c.eps, (info, err)
        assert abs(err - info["rel_err"]) <= 1e-3 * c.eps + 1e-14
        if info["row_first"] < info["col_first"]:      # the compressed one of the pair
            if Q.shape[1]:
                ortho = float(np.max(np.abs(Q.conj().T @ Q - np.eye(Q.shape[1]))))
                assert ortho <= 1e-12, (info, ortho)
            mir = by_key[(tuple(cols), tuple(rows))]
            assert np.array_equal(mir[2], R.T) and np.array_equal(mir[3], Q.T)
            mirror_checked += 1
    assert mirror_checked == len(c.factors()) // 2


def test_ranks_close_to_the_svd_bound():
    """Pivoted-QR ranks are near the Eckart-Young minimum (tiny: QRCP ~ 1.09 x SVD)."""
    c = case("tiny")
    ratios = []
    for rows, cols, Q, R, info in c.factors()[:40]:
        B = greens.assemble_block(c.disc, rows, cols)
        r_svd = compressed.svd_rank(B, c.eps)
        assert Q.shape[1] >= r_svd
        ratios.append(Q.shape[1] / max(r_svd, 1))
    assert np.mean(ratios) < 1.3


@pytest.mark.parametrize("name", NAMES)
def test_apply_matches_oracle_on_the_same_factors_and_bounds_dense(name):
    c = case(name)
    n = c.geom.ndof
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    y = to_host(c.op.apply(to_dev(x)))
    sb = greens.self_blocks(c.disc)
    fac = [(f[0], f[1], f[2], f[3]) for f in c.factors()]
    for r in range(2):
        ref = compressed.compressed_apply(sb, fac, x[r])
        assert np.linalg.norm(y[r] - ref) <= 1e-12 * np.linalg.norm(ref)
        Zx = c.Z @ x[r]
        Zoff = c.Z.copy()
        for p in range(c.array.n_particles):
            Zoff[p * 144:(p + 1) * 144, p * 144:(p + 1) * 144] = 0
        assert np.linalg.norm(y[r] - Zx) <= c.eps * np.linalg.norm(Zoff) * np.linalg.norm(x[r])


@pytest.mark.parametrize("nrhs", [2, 3, 8, 11])
def test_multi_rhs_apply_matches_the_oracle(nrhs):
    """Blocks of right-hand sides stream each factor once for the whole block."""
    c = case("rand6x7")
    n = c.geom.ndof
    rng = np.random.default_rng(nrhs)
    x = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    y = to_host(c.op.apply(to_dev(x)))
    sb = greens.self_blocks(c.disc)
    fac = [(f[0], f[1], f[2], f[3]) for f in c.factors()]
    ref = compressed.compressed_apply(sb, fac, x.T).T
    for r in range(nrhs):
        assert np.linalg.norm(y[r] - ref[r]) <= 1e-12 * np.linalg.norm(ref[r])


@pytest.mark.parametrize("name,nrhs", [("rand6x7", 16), ("rand6x7", 37), ("rand5x3", 64), ("rand6x7", 70)])
def test_block_apply_matches_the_oracle(name, nrhs):
    """16 or more right-hand sides run on the FP64 MFMA strip kernels, 64 per block."""
    c = case(name)
    n = c.geom.ndof
    rng = np.random.default_rng(100 + nrhs)
    x = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    y = to_host(c.op.apply(to_dev(x)))
    sb = greens.self_blocks(c.disc)
    fac = [(f[0], f[1], f[2], f[3]) for f in c.factors()]
    ref = compressed.compressed_apply(sb, fac, x.T).T
    for r in range(nrhs):
        assert np.linalg.norm(y[r] - ref[r]) <= 1e-12 * np.linalg.norm(ref[r])
    # a column's result does not depend on the other columns of its block
    y1 = to_host(c.op.apply(to_dev(x[nrhs - 1:nrhs])))
    assert np.linalg.norm(y1[0] - y[nrhs - 1]) <= 1e-13 * np.linalg.norm(y1[0])


def test_grouped_solve_matches_lu_for_every_rhs():
    """Up to eight right-hand sides advance together and share each product (§8 a8)."""
    import paper_2603_10586_amd as q
    c = case("rand6x7")
    th = np.linspace(-30, 30, 5)
    v = q.rhs_plane_waves(c.ctx, c.geom, np.concatenate([th, th]), np.zeros(10), [0] * 5 + [1] * 5)
    x, info, st = c.op.solve(v, restart=60, tol=1e-10, max_iter=3000)
    assert st == 0 and all(i["converged"] for i in info)
    sb = greens.self_blocks(c.disc)
    ZQR = compressed.dense_from_factors(sb, [(f[0], f[1], f[2], f[3]) for f in c.factors()])
    vh, xh = to_host(v), to_host(x)
    ref = np.linalg.solve(ZQR, vh.T).T
    for r in range(10):
        assert np.linalg.norm(xh[r] - ref[r]) <= 1e-8 * np.linalg.norm(ref[r])
    # each column alone gives the same solution (to the solver tolerance)
    x1, info1, _ = c.op.solve(v[3:4].contiguous(), restart=60, tol=1e-10, max_iter=3000)
    assert np.linalg.norm(to_host(x1)[0] - xh[3]) <= 1e-8 * np.linalg.norm(xh[3])


def test_apply_is_bitwise_reproducible():
    c = case("rand6x7")
    x = to_dev(np.random.default_rng(9).standard_normal(c.geom.ndof) + 0.5j)
    a = to_host(c.op.apply(x))
    b = to_host(c.op.apply(x))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name", NAMES)
def test_precondition_matches_oracle(name):
    c = case(name)
    y = np.random.default_rng(4).standard_normal(c.geom.ndof) * (1 - 2j)
    z = to_host(c.op.precondition(to_dev(y)))
    P = solvers.BlockDiagPreconditioner(greens.self_blocks(c.disc))
    ref = P.apply(y)
    assert np.linalg.norm(z - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", NAMES)
def test_solve_matches_lu_of_the_same_operator(name):
    """F1: GPU GMRES vs the oracle's direct solve of the exported Z_QR."""
    import paper_2603_10586_amd as q
    c = case(name)
    v = q.rhs_plane_waves(c.ctx, c.geom, [0.0, 20.0], [0.0, 0.0], [1, 0])
    x, info, st = c.op.solve(v, restart=30, tol=1e-10, max_iter=2000)
    assert st == 0 and all(i["converged"] for i in info)
    sb = greens.self_blocks(c.disc)
    ZQR = compressed.dense_from_factors(sb, [(f[0], f[1], f[2], f[3]) for f in c.factors()])
    vh = to_host(v)
    xh = to_host(x)
    for r in range(2):
        ref = np.linalg.solve(ZQR, vh[r])
        assert np.linalg.norm(xh[r] - ref) <= 1e-6 * np.linalg.norm(ref)
        assert info[r]["rel_res_true"] <= 1e-10


@pytest.mark.parametrize("restart", [7, 40, 4096])
def test_solve_is_independent_of_the_restart_length(restart):
    """Short restarts, mid-cycle acceptance and unrestarted runs reach the same solution."""
    import paper_2603_10586_amd as q
    c = case("rand6x7")
    v = q.rhs_plane_waves(c.ctx, c.geom, [5.0], [0.0], [0])
    x, info, st = c.op.solve(v, restart=restart, tol=1e-10, max_iter=4000)
    assert st == 0 and info[0]["converged"] and info[0]["rel_res_true"] <= 1e-10
    sb = greens.self_blocks(c.disc)
    ZQR = compressed.dense_from_factors(sb, [(f[0], f[1], f[2], f[3]) for f in c.factors()])
    ref = np.linalg.solve(ZQR, to_host(v)[0])
    assert np.linalg.norm(to_host(x)[0] - ref) <= 1e-8 * np.linalg.norm(ref)
    if restart >= 4096:
        assert info[0]["restarts"] == 0          # accepted inside the first Krylov space


def test_solve_reports_not_converged_with_the_best_iterate():
    import paper_2603_10586_amd as q
    c = case("rand6x7")
    v = q.rhs_plane_waves(c.ctx, c.geom, [0.0], [0.0], [1])
    x, info, st = c.op.solve(v, restart=30, tol=1e-12, max_iter=5)
    assert st == 5 and not info[0]["converged"] and info[0]["iterations"] == 5
    assert 0 < info[0]["rel_res_true"] < 1.0


def test_solve_method_accuracy_against_uncompressed_lu():
    """F3 on the tiny array: eps_sol within 3x the oracle's own QRCP compression."""
    import paper_2603_10586_amd as q
    c = case("tiny")
    v = q.rhs_plane_waves(c.ctx, c.geom, [0.0], [0.0], [1])
    x, info, st = c.op.solve(v, restart=30, tol=1e-8)
    xh = to_host(x)[0]
    x_lu = np.linalg.solve(c.Z, to_host(v)[0])
    eps_sol = np.linalg.norm(xh - x_lu) / np.linalg.norm(x_lu)
    fac = []
    for b in c.oracle_blocks():
        B = greens.assemble_block(c.disc, b.rows, b.cols)
        Q, R = compressed.qrcp_truncate(B, c.eps)
        fac.append((b.rows, b.cols, Q, R))
    ZQR_o = compressed.dense_from_factors(greens.self_blocks(c.disc), fac)
    eps_sol_o = np.linalg.norm(np.linalg.solve(ZQR_o, to_host(v)[0]) - x_lu) / np.linalg.norm(x_lu)
    assert eps_sol <= 3 * max(eps_sol_o, 1e-7), (eps_sol, eps_sol_o)


def test_tighter_eps_gives_accurate_solution():
    """eps = 1e-9: the compressed solution meets 1e-6 against the uncompressed LU outright."""
    import paper_2603_10586_amd as q
    c = case("tiny", eps=1e-9)
    v = q.rhs_plane_waves(c.ctx, c.geom, [0.0], [0.0], [1])
    x, info, st = c.op.solve(v, restart=30, tol=1e-10)
    x_lu = np.linalg.solve(c.Z, to_host(v)[0])
    assert np.linalg.norm(to_host(x)[0] - x_lu) <= 1e-6 * np.linalg.norm(x_lu)


def test_gain_and_stats_are_consistent():
    c = case("rand6x7")
    s = c.op.stats()
    n = c.geom.ndof
    nqr = c.array.n_particles * 144 * 144 + sum((f[4]["m"] + f[4]["n"]) * f[4]["rank"] for f in c.factors())
    assert s["n_qr_entries"] == nqr
    assert abs(s["gain"] - n * n / nqr) <= 1e-12 * s["gain"]
    assert s["max_block_rel_err"] <= c.eps
    assert s["n_blocks"] == len(c.factors())


def test_factors_do_not_depend_on_the_compression_chunking():
    """Sketches are seeded per block and every reduction has a fixed order, so compressing
    the blocks in small chunks (several launches, retries per chunk) gives bitwise the
    factors of one large chunk (§5.2 compression, scheduled in chunks of device memory)."""
    import paper_2603_10586_amd as q
    c = case("rand8x8")
    small = q.Operator(c.ctx, c.geom, eps=c.eps, chunk_bytes=8 << 20)
    assert small.num_blocks() == c.op.num_blocks()
    for b in range(small.num_blocks()):
        i1, Q1, R1 = small.export_block(b)
        i0, Q0, R0 = c.op.export_block(b)
        assert i1 == i0
        if Q0 is None:
            assert Q1 is None
            continue
        assert np.array_equal(Q1, Q0) and np.array_equal(R1, R0)
    with pytest.raises(q.QrvieError):
        q.Operator(c.ctx, c.geom, eps=c.eps, chunk_bytes=-1)


def test_read_probe_reports_a_rate_below_the_hbm_peak():
    import torch
    import paper_2603_10586_amd as q
    c = case("tiny")
    buf = torch.ones(1 << 25, dtype=torch.float64, device="cuda")        # 256 MiB
    gbs = c.ctx.probe_read(buf, reps=2)
    assert 100.0 < gbs < 8000.0
    with pytest.raises(q.QrvieError):
        c.ctx.check(c.ctx.lib.qrvie_probe_read(c.ctx.h, None, 16, 1, None), "probe")


def test_matrix_core_probe_reports_plausible_rates():
    c = case("tiny")
    f64, f32 = c.ctx.probe_mfma(True), c.ctx.probe_mfma(False)
    assert 5.0 < f64 < 200.0 and 5.0 < f32 < 400.0


def test_edge_blocks_of_an_odd_lattice_compress():
    """A 33 x 33 lattice has one-particle nodes at its edge, so it has tall far blocks of one
    particle's columns (2304 x 144) whose sketch is retried at full width; every block must
    still be certified (a GEMM variant that failed here is not used)."""
    import paper_2603_10586_amd as q
    import workloads as W
    arr = W.serving_requests(n=8, seed=0, rate_per_s=1.0, side_lo=8, side_hi=48)[7].array
    assert arr.n_particles == 1089
    c = case("tiny")
    geom = q.Geometry(c.ctx, arr)
    op = q.Operator(c.ctx, geom, eps=1e-6, max_block_rows=9216)
    assert op.num_blocks() == 42714
    worst = max(op.export_block(b, factors=False)[0]["rel_err"] for b in range(op.num_blocks()))
    assert worst <= 1e-6
