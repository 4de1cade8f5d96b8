"""Reduced-precision far factors and mixed-precision iterative refinement (GPU).

The complex64 operator Z_lo is defined exactly: the self blocks in complex128 and each
far factor rounded to nearest complex64, with every product accumulated in FP64.  The
oracle therefore evaluates Z_lo x from the exported complex128 factors rounded by numpy
(both sides round to nearest-even), and the two agree to FP64 accumulation order
(1e-12 relative).  Refinement must reach the true residual of the complex128 operator
Z_QR: solutions are compared with the oracle's LU of the exported Z_QR.
"""
import numpy as np
import pytest

from oracle import compressed, greens

from gpu_cases import case, to_dev, to_host

pytestmark = pytest.mark.gpu

PREC_C64 = 1
MIXED_IR = 1


def _lo_factors(c):
    return [(f[0], f[1], f[2].astype(np.complex64).astype(np.complex128),
             f[3].astype(np.complex64).astype(np.complex128)) for f in c.factors()]


@pytest.mark.parametrize("nrhs", [1, 3, 8])
def test_c64_product_matches_the_oracle_on_rounded_factors(nrhs):
    c = case("rand6x7", far_prec=PREC_C64)
    n = c.geom.ndof
    rng = np.random.default_rng(40 + nrhs)
    x = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    y = to_host(c.op.apply(to_dev(x), prec=PREC_C64))
    sb = greens.self_blocks(c.disc)
    ref = compressed.compressed_apply(sb, _lo_factors(c), x.T).T
    for r in range(nrhs):
        assert np.linalg.norm(y[r] - ref[r]) <= 1e-12 * np.linalg.norm(ref[r])


def test_c64_product_differs_from_c128_by_the_factor_rounding_only():
    c = case("rand6x7", far_prec=PREC_C64)
    x = to_dev(np.random.default_rng(7).standard_normal(c.geom.ndof) * (1 + 1j))
    hi = to_host(c.op.apply(x))
    lo = to_host(c.op.apply(x, prec=PREC_C64))
    d = np.linalg.norm(lo - hi) / np.linalg.norm(hi)
    assert 0.0 < d <= 1e-6        # complex64 rounding is 6e-8 per entry


def test_c128_product_of_a_c64_operator_is_unchanged():
    """Building the complex64 copy leaves the complex128 factors and product untouched."""
    c = case("rand6x7", far_prec=PREC_C64)
    x = np.random.default_rng(8).standard_normal(c.geom.ndof) + 0.25j
    y = to_host(c.op.apply(to_dev(x)))
    sb = greens.self_blocks(c.disc)
    ref = compressed.compressed_apply(sb, [(f[0], f[1], f[2], f[3]) for f in c.factors()], x)
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("name,nrhs", [("rand5x3", 1), ("rand6x7", 3), ("rand6x7", 10)])
def test_mixed_ir_reaches_the_c128_solution(name, nrhs):
    import paper_2603_10586_amd as q
    c = case(name, far_prec=PREC_C64)
    th = np.linspace(-40, 40, nrhs)
    v = q.rhs_plane_waves(c.ctx, c.geom, th, np.zeros(nrhs), [r % 2 for r in range(nrhs)])
    x, info, st = c.op.solve(v, restart=500, tol=1e-10, max_iter=4000, mode=MIXED_IR)
    assert st == 0
    sb = greens.self_blocks(c.disc)
    ZQR = compressed.dense_from_factors(sb, [(f[0], f[1], f[2], f[3]) for f in c.factors()])
    vh, xh = to_host(v), to_host(x)
    ref = np.linalg.solve(ZQR, vh.T).T
    for r in range(nrhs):
        assert info[r]["converged"] and info[r]["rel_res_true"] <= 1e-10
        assert info[r]["n_refine"] >= 1
        res = np.linalg.norm(vh[r] - ZQR @ xh[r]) / np.linalg.norm(vh[r])
        assert res <= 2e-10                       # true residual of Z_QR, recomputed by the oracle
        assert np.linalg.norm(xh[r] - ref[r]) <= 1e-7 * np.linalg.norm(ref[r])


def test_mixed_ir_at_the_working_tolerance_needs_few_refinements():
    import paper_2603_10586_amd as q
    c = case("rand8x8", far_prec=PREC_C64)
    v = q.rhs_plane_waves(c.ctx, c.geom, [10.0], [0.0], [1])
    x, info, st = c.op.solve(v, restart=1000, tol=1e-6, max_iter=2000, mode=MIXED_IR)
    x64, info64, st64 = c.op.solve(v, restart=1000, tol=1e-6, max_iter=2000)
    assert st == 0 and st64 == 0
    assert 1 <= info[0]["n_refine"] <= 3
    assert info[0]["rel_res_true"] <= 1e-6
    assert info64[0]["n_refine"] == 0
    d = np.linalg.norm(to_host(x) - to_host(x64)) / np.linalg.norm(to_host(x64))
    assert d <= 1e-4                               # both within tol of the same system


def test_reduced_precision_requests_without_a_c64_copy_are_refused():
    import paper_2603_10586_amd as q
    c = case("rand5x3")
    v = q.rhs_plane_waves(c.ctx, c.geom, [0.0], [0.0], [1])
    with pytest.raises(q.QrvieError) as e:
        c.op.solve(v, mode=MIXED_IR)
    assert e.value.status == 1
    with pytest.raises(q.QrvieError) as e:
        c.op.apply(v, prec=PREC_C64)
    assert e.value.status == 1


C64_ONLY = 3


@pytest.mark.parametrize("nrhs", [1, 3, 16, 37])
def test_c64_only_operator_products_match_the_oracle(nrhs):
    """Only complex64 panels are kept; every product path (single, grouped, MFMA block)
    uses them, and exports return those values widened."""
    c = case("rand6x7", far_prec=C64_ONLY)
    n = c.geom.ndof
    rng = np.random.default_rng(60 + nrhs)
    x = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    y = to_host(c.op.apply(to_dev(x)))
    sb = greens.self_blocks(c.disc)
    ref = compressed.compressed_apply(sb, [(f[0], f[1], f[2], f[3]) for f in c.factors()], x.T).T
    for r in range(nrhs):
        assert np.linalg.norm(y[r] - ref[r]) <= 1e-12 * np.linalg.norm(ref[r])


def test_c64_only_panels_equal_the_rounded_complex128_panels():
    """The same compression packed straight to complex64 gives the copy's values exactly."""
    a = case("rand6x7", far_prec=C64_ONLY)
    b = case("rand6x7", far_prec=PREC_C64)
    x = to_dev(np.random.default_rng(70).standard_normal(a.geom.ndof) * (1 - 1j))
    assert np.array_equal(to_host(a.op.apply(x)), to_host(b.op.apply(x, prec=PREC_C64)))
    assert a.op.stats()["device_bytes"] < b.op.stats()["device_bytes"]


@pytest.mark.parametrize("mode", [0, 2])
def test_c64_only_solves_match_lu_of_the_stored_operator(mode):
    import paper_2603_10586_amd as q
    c = case("rand6x7", far_prec=C64_ONLY)
    th = np.linspace(-30, 30, 6)
    v = q.rhs_plane_waves(c.ctx, c.geom, th, np.zeros(6), [0, 1] * 3)
    x, info, st = c.op.solve(v, restart=500, tol=1e-10, max_iter=2000, mode=mode)
    assert st == 0 and all(i["converged"] for i in info)
    sb = greens.self_blocks(c.disc)
    ZQR = compressed.dense_from_factors(sb, [(f[0], f[1], f[2], f[3]) for f in c.factors()])
    vh, xh = to_host(v), to_host(x)
    ref = np.linalg.solve(ZQR, vh.T).T
    for r in range(6):
        assert np.linalg.norm(xh[r] - ref[r]) <= 1e-7 * np.linalg.norm(ref[r])


def test_c64_only_refuses_complex128_requests():
    import paper_2603_10586_amd as q
    c = case("rand6x7", far_prec=C64_ONLY)
    v = q.rhs_plane_waves(c.ctx, c.geom, [0.0], [0.0], [1])
    with pytest.raises(q.QrvieError) as e:
        c.op.solve(v, mode=MIXED_IR)
    assert e.value.status == 1
    with pytest.raises(q.QrvieError) as e:
        c.op.apply(v, prec=0)
    assert e.value.status == 1


BLOCK_IR = 3


@pytest.mark.parametrize("name,nrhs", [("rand5x3", 1), ("rand6x7", 10), ("rand6x7", 70)])
def test_block_ir_reaches_the_c128_solution(name, nrhs):
    """Refinement with block corrections on the complex64 panels: every column's true
    residual of Z_QR (complex128 factors, recomputed by the oracle) meets tol."""
    import paper_2603_10586_amd as q
    c = case(name, far_prec=PREC_C64)
    rng = np.random.default_rng(nrhs)
    th = rng.uniform(-40, 40, nrhs)
    v = q.rhs_plane_waves(c.ctx, c.geom, th, rng.uniform(0, 360, nrhs), [r % 2 for r in range(nrhs)])
    x, info, st = c.op.solve(v, restart=4000, tol=1e-10, max_iter=2000, mode=BLOCK_IR)
    assert st == 0
    sb = greens.self_blocks(c.disc)
    ZQR = compressed.dense_from_factors(sb, [(f[0], f[1], f[2], f[3]) for f in c.factors()])
    vh, xh = to_host(v), to_host(x)
    ref = np.linalg.solve(ZQR, vh.T).T
    for r in range(nrhs):
        assert info[r]["converged"] and info[r]["rel_res_true"] <= 1e-10
        assert info[r]["n_refine"] >= 1
        res = np.linalg.norm(vh[r] - ZQR @ xh[r]) / np.linalg.norm(vh[r])
        assert res <= 2e-10
        assert np.linalg.norm(xh[r] - ref[r]) <= 1e-7 * np.linalg.norm(ref[r])


def test_block_ir_matches_block_fp64_at_the_working_tolerance():
    import paper_2603_10586_amd as q
    c = case("rand8x8", far_prec=PREC_C64)
    th = np.linspace(-30, 30, 8)
    v = q.rhs_plane_waves(c.ctx, c.geom, th, np.zeros(8), [r % 2 for r in range(8)])
    x, info, st = c.op.solve(v, restart=4000, tol=1e-6, max_iter=2000, mode=BLOCK_IR)
    x64, info64, st64 = c.op.solve(v, restart=4000, tol=1e-6, max_iter=2000, mode=q.SOLVE_BLOCK)
    assert st == 0 and st64 == 0
    xh, x64h = to_host(x), to_host(x64)
    for r in range(8):
        assert info[r]["rel_res_true"] <= 1e-6 and 1 <= info[r]["n_refine"] <= 3
        assert np.linalg.norm(xh[r] - x64h[r]) <= 1e-4 * np.linalg.norm(x64h[r])


def test_block_ir_needs_the_c64_copy():
    import paper_2603_10586_amd as q
    c = case("rand5x3")
    v = q.rhs_plane_waves(c.ctx, c.geom, [0.0], [0.0], [1])
    with pytest.raises(q.QrvieError) as e:
        c.op.solve(v, mode=BLOCK_IR)
    assert e.value.status == 1
