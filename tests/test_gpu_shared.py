"""Transpose-shared factor storage against the oracle and against per-block storage.

Z is complex symmetric (the symmetric weak form, §2 eq. 2.5), so the mirror block (J, I) of
a far pair is the transpose of (I, J): with ``share_transpose`` the library keeps one Q, R per
pair and applies the mirror as R^T (Q^T x_I).  Compression does not depend on the storage,
so a shared operator holds bitwise the factors of the unshared one, and its products differ
only by summation order (1e-12 relative); against the oracle's product of the exported
factors the bar is the same accumulated FP64 rounding.
"""
import numpy as np
import pytest

from oracle import compressed, greens

from gpu_cases import ARRAYS, case, ctx, mid, to_dev, to_host

pytestmark = pytest.mark.gpu

_SH = {}


def shared(name, far_prec=0):
    key = (name, far_prec)
    if key not in _SH:
        import paper_2603_10586_amd as q
        c = case(name, far_prec=far_prec)
        print(f"[gpu case] shared operator {name} far_prec={far_prec}", flush=True)
        _SH[key] = q.Operator(c.ctx, c.geom, eps=c.eps, far_prec=far_prec, share_transpose=True)
    return _SH[key]


@pytest.mark.parametrize("name", ["tiny", "rand5x3", "rand6x7"])
def test_shared_factors_equal_the_unshared_factors(name):
    c = case(name)
    op = shared(name)
    assert op.num_blocks() == c.op.num_blocks()
    for b in range(op.num_blocks()):
        i1, Q1, R1 = op.export_block(b)
        i0, Q0, R0 = c.op.export_block(b)
        assert i1 == i0
        if Q0 is None:
            assert Q1 is None
        else:
            assert np.array_equal(Q1, Q0) and np.array_equal(R1, R0)


@pytest.mark.parametrize("name", ["tiny", "rand5x3", "rand6x7"])
def test_shared_product_matches_the_oracle_and_the_unshared_product(name):
    c = case(name)
    op = shared(name)
    n = c.geom.ndof
    rng = np.random.default_rng(50)
    x = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    y = to_host(op.apply(to_dev(x)))
    y0 = to_host(c.op.apply(to_dev(x)))
    sb = greens.self_blocks(c.disc)
    fac = [(f[0], f[1], f[2], f[3]) for f in c.factors()]
    for r in range(3):
        ref = compressed.compressed_apply(sb, fac, x[r])
        assert np.linalg.norm(y[r] - ref) <= 1e-12 * np.linalg.norm(ref)
        assert np.linalg.norm(y[r] - y0[r]) <= 1e-12 * np.linalg.norm(y0[r])
    y1 = to_host(op.apply(to_dev(x[1])))                     # one column alone: the same product
    assert np.array_equal(y1, y[1])


def test_shared_product_is_complex_symmetric_and_reproducible():
    c = case("rand6x7")
    op = shared("rand6x7")
    rng = np.random.default_rng(51)
    n = c.geom.ndof
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    Zx, Zv = to_host(op.apply(to_dev(x))), to_host(op.apply(to_dev(v)))
    assert abs(x @ Zv - v @ Zx) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(Zv)
    assert np.array_equal(to_host(op.apply(to_dev(x))), Zx)


def test_shared_storage_halves_the_factor_memory_and_the_streamed_bytes():
    c = case("rand6x7")
    op = shared("rand6x7")
    s0, s1 = c.op.stats(), op.stats()
    self_bytes = 2 * s0["n_self_types"] * 144 * 144 * 16
    assert s1["n_qr_entries"] == s0["n_qr_entries"]
    assert (s1["device_bytes"] - self_bytes) <= 0.55 * (s0["device_bytes"] - self_bytes)
    assert s1["apply_bytes"] < 0.8 * s0["apply_bytes"]
    prof = op.profile_apply(reps=2)
    total = sum(prof[k]["bytes"] for k in ("rphase", "qphase", "final", "qtphase"))
    assert prof["product"]["bytes"] == total == s1["apply_bytes"]
    assert prof["qtphase"]["ms"] > 0.0


@pytest.mark.parametrize("name", ["tiny", "rand6x7"])
def test_shared_solve_matches_lu_of_the_same_operator(name):
    """F1 on the shared operator: FP64 GMRES, and mixed-precision refinement on its complex64 copy."""
    import paper_2603_10586_amd as q
    c = case(name)
    sb = greens.self_blocks(c.disc)
    ZQR = compressed.dense_from_factors(sb, [(f[0], f[1], f[2], f[3]) for f in c.factors()])
    v = q.rhs_plane_waves(c.ctx, c.geom, [0.0, 20.0], [0.0, 0.0], [1, 0])
    vh = to_host(v)
    for far_prec, mode in ((0, q.SOLVE_FP64), (1, q.SOLVE_MIXED_IR)):
        op = shared(name, far_prec)
        x, info, st = op.solve(v, restart=60, tol=1e-10, max_iter=3000, mode=mode)
        assert st == 0 and all(i["converged"] for i in info)
        xh = to_host(x)
        for r in range(2):
            ref = np.linalg.solve(ZQR, vh[r])
            assert np.linalg.norm(xh[r] - ref) <= 1e-8 * np.linalg.norm(ref)


def test_shared_operator_refuses_the_block_tuner_and_stage_profiler():
    """Block solves take shared operators (test_gpu_lowprec.py); the tile autotuner and the
    block-product stage profiler time per-block storage only."""
    import paper_2603_10586_amd as q
    shared("rand6x7")
    op = shared("rand6x7")
    with pytest.raises(q.QrvieError):
        op.tune_block(nrhs=16)
    with pytest.raises(q.QrvieError):
        op.profile_block(nrhs=16)


def test_shared_many_rhs_products_equal_single_products():
    """2-15 right-hand sides: one single-RHS product per column (bitwise); 16 or more: the block
    product with Q^T and R^T strips (accumulated FP64 rounding)."""
    c = case("rand5x3")
    op = shared("rand5x3")
    rng = np.random.default_rng(52)
    x = rng.standard_normal((20, c.geom.ndof)) + 0.5j
    y5 = to_host(op.apply(to_dev(x[:5])))
    y20 = to_host(op.apply(to_dev(x)))
    for r in (0, 4):
        one = to_host(op.apply(to_dev(x[r])))
        assert np.array_equal(y5[r], one)
        assert np.linalg.norm(y20[r] - one) <= 1e-12 * np.linalg.norm(one)


def test_shared_full_size_product_matches_the_unshared_product():
    """Mid-size (32 x 32): the shared product against the per-block-storage product (whose rows
    are checked against the oracle in the full-size tests) and its symmetry."""
    import paper_2603_10586_amd as q
    m = mid()
    op = q.Operator(ctx(), m["geom"], eps=1e-6, share_transpose=True)
    n = m["geom"].ndof
    rng = np.random.default_rng(53)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = to_host(op.apply(to_dev(x)))
    y0 = to_host(m["op"].apply(to_dev(x)))
    # the same factors summed in another order: every entry is a sum of at most n products, so
    # two FP64 orders differ by at most 2 gamma_n (n u each) times the sum of the products'
    # magnitudes; bounded here by 8 n u ||y0|| (measured: 3.3e-11 relative, about 2 n u)
    u = 2.0 ** -53
    assert np.linalg.norm(y - y0) <= 8 * n * u * np.linalg.norm(y0)
    Zv = to_host(op.apply(to_dev(v)))
    assert abs(x @ Zv - v @ y) <= 8 * n * u * np.linalg.norm(x) * np.linalg.norm(Zv)
    s0, s1 = m["op"].stats(), op.stats()
    print(f"[shared mid] device GB {s1['device_bytes'] / 1e9:.2f} vs {s0['device_bytes'] / 1e9:.2f}, "
          f"product GB {s1['apply_bytes'] / 1e9:.2f} vs {s0['apply_bytes'] / 1e9:.2f}", flush=True)
    op.close()
