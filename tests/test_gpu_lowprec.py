"""Block products on transpose-shared factors and on FP32 matrix cores, and the refinement
modes built on them (GPU against the oracle).

* Shared factors in block products: the Q^T and R^T strips apply each mirror block as
  R^T (Q^T X) on FP64 matrix cores; the oracle's product of the exported factors agrees to
  accumulated FP64 rounding (1e-12).
* FP32 matrix cores (QRVIE_PREC_C64_F32: complex64 far factors and self blocks; and
  QRVIE_PREC_BF16X2: BF16 split-complex far factors, complex64 self blocks): the operator is
  defined exactly by the rounded factors, and the product accumulates in FP32 with the
  right-hand sides rounded to FP32.  The oracle evaluates the same rounded operator in FP64
  (BF16 rounding written out from its definition: round to nearest even on the FP32 bit
  pattern, after FP64 -> FP32), and each output must lie within the standard bound of
  floating-point inner products, gamma_K (|Z_lo| |x|)_i with gamma_K = 2 (K + 2) u, u = 2^-24,
  K the longest accumulation (a panel strip's columns plus a rank sum).
* Refinement with these corrections must reach the solution of its residual operator to the
  solver tolerance: compared with the oracle's LU of that operator.
"""
import numpy as np
import pytest

from oracle import compressed, greens

from gpu_cases import case, to_dev, to_host

pytestmark = pytest.mark.gpu

PREC_C64, PREC_BF16X2, PREC_C64_ONLY, PREC_C64_F32 = 1, 2, 3, 4
U32 = 2.0 ** -24


def _factors(c):
    return [(f[0], f[1], f[2], f[3]) for f in c.factors()]


def _bf16(z):
    """Round complex values to BF16 parts: FP64 -> FP32 (nearest even), then the FP32 bit
    pattern to its upper 16 bits, round to nearest even."""
    def part(a):
        u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
        h = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF
        return (h.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return part(z.real) + 1j * part(z.imag)


def _c64(z):
    return np.asarray(z).astype(np.complex64).astype(np.complex128)


def _abs_product(sb, fac, x):
    """(|Z_D| |x| + sum |Q| (|R| |x|)), the magnitudes an inner-product error bound scales with."""
    ax = np.abs(x)
    return compressed.compressed_apply(np.abs(sb), [(r, c, np.abs(Q), np.abs(R)) for r, c, Q, R in fac], ax)


def _kmax(c):
    """Longest FP32 accumulation of the product, in terms: the widest block (a strip's columns
    in the R and Q^T passes, the self block) plus the largest rank sum of a row or column node
    (the Q and R^T passes); a complex multiply-add counts as two real terms."""
    infos = [f[4] for f in c.factors()]
    sums = {}
    for i in infos:
        for key in (("r", i["level"], i["row_first"]), ("c", i["level"], i["col_first"])):
            sums[key] = sums.get(key, 0) + i["rank"]
    return 2 * (max(max(i["n"] for i in infos), 144) + max(sums.values()))


@pytest.mark.parametrize("name,nrhs", [("rand6x7", 16), ("rand6x7", 37), ("rand5x3", 70)])
def test_shared_block_product_matches_the_oracle(name, nrhs):
    import paper_2603_10586_amd as q
    c = case(name)
    op = q.Operator(c.ctx, c.geom, eps=c.eps, share_transpose=True)
    n = c.geom.ndof
    rng = np.random.default_rng(60 + nrhs)
    x = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    y = to_host(op.apply(to_dev(x)))
    ref = compressed.compressed_apply(greens.self_blocks(c.disc), _factors(c), x.T).T
    for r in range(nrhs):
        assert np.linalg.norm(y[r] - ref[r]) <= 1e-12 * np.linalg.norm(ref[r])
    op.close()


def test_shared_block_solve_matches_lu_of_the_same_operator():
    import paper_2603_10586_amd as q
    c = case("rand6x7")
    op = q.Operator(c.ctx, c.geom, eps=c.eps, share_transpose=True)
    th = np.linspace(-30, 30, 5)
    v = q.rhs_plane_waves(c.ctx, c.geom, np.concatenate([th, th]), np.zeros(10), [0] * 5 + [1] * 5)
    x, info, st = op.solve(v, restart=2000, tol=1e-10, max_iter=2000, mode=q.SOLVE_BLOCK)
    assert st == 0 and all(i["converged"] for i in info)
    ZQR = compressed.dense_from_factors(greens.self_blocks(c.disc), _factors(c))
    vh, xh = to_host(v), to_host(x)
    ref = np.linalg.solve(ZQR, vh.T).T
    for r in range(10):
        assert np.linalg.norm(xh[r] - ref[r]) <= 1e-8 * np.linalg.norm(ref[r])
    op.close()


@pytest.mark.parametrize("shared", [False, True])
@pytest.mark.parametrize("nrhs", [1, 8, 20])
def test_fp32_product_of_complex64_factors_meets_the_inner_product_bound(nrhs, shared):
    import paper_2603_10586_amd as q
    c = case("rand6x7", far_prec=PREC_C64)
    op = q.Operator(c.ctx, c.geom, eps=c.eps, far_prec=PREC_C64, share_transpose=True) if shared else c.op
    n = c.geom.ndof
    rng = np.random.default_rng(70 + nrhs)
    x = rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))
    y = to_host(op.apply(to_dev(x), prec=PREC_C64_F32))
    sb = _c64(greens.self_blocks(c.disc))
    fac = [(r, cc, _c64(Q), _c64(R)) for r, cc, Q, R in _factors(c)]
    ref = compressed.compressed_apply(sb, fac, x.T).T
    mag = _abs_product(sb, fac, x.T).T
    gamma = 2 * (_kmax(c) + 4) * U32
    for r in range(nrhs):
        assert np.all(np.abs(y[r] - ref[r]) <= gamma * mag[r])
        assert np.linalg.norm(y[r] - ref[r]) > 0.0                       # FP32, not FP64, arithmetic
    if shared:
        op.close()


@pytest.mark.parametrize("shared", [False, True])
def test_bf16_product_meets_the_inner_product_bound(shared):
    import paper_2603_10586_amd as q
    c = case("rand6x7")
    op = q.Operator(c.ctx, c.geom, eps=c.eps, far_prec=PREC_BF16X2, share_transpose=shared)
    n = c.geom.ndof
    rng = np.random.default_rng(80)
    x = rng.standard_normal((8, n)) + 1j * rng.standard_normal((8, n))
    y = to_host(op.apply(to_dev(x), prec=PREC_BF16X2))
    sb = _c64(greens.self_blocks(c.disc))
    fac = [(r, cc, _bf16(Q), _bf16(R)) for r, cc, Q, R in _factors(c)]
    ref = compressed.compressed_apply(sb, fac, x.T).T
    mag = _abs_product(sb, fac, x.T).T
    gamma = 2 * (_kmax(c) + 4) * U32
    for r in range(8):
        assert np.all(np.abs(y[r] - ref[r]) <= gamma * mag[r])
    # the BF16 operator differs from the complex128 one by its rounding (2^-9 relative per entry)
    y64 = to_host(c.op.apply(to_dev(x)))
    d = np.linalg.norm(y - y64) / np.linalg.norm(y64)
    assert 1e-5 < d < 2e-2
    # the operator's own (complex64) factors are exported, and its plain products use them
    yc = to_host(op.apply(to_dev(x[:1])))
    fac64 = [(r, cc, _c64(Q), _c64(R)) for r, cc, Q, R in _factors(c)]
    ref64 = compressed.compressed_apply(greens.self_blocks(c.disc), fac64, x[0])
    assert np.linalg.norm(yc[0] - ref64) <= 1e-12 * np.linalg.norm(ref64)
    op.close()


def _lu_reference(c, factors, v):
    Z = compressed.dense_from_factors(greens.self_blocks(c.disc), factors)
    return np.linalg.solve(Z, v.T).T


@pytest.mark.parametrize("shared", [False, True])
def test_bf16_block_refinement_reaches_its_operator_solution(shared):
    """The precision pattern on a small array: BF16 corrections on FP32 matrix cores, FP64
    residuals of the complex64 operator, 8 plane waves."""
    import paper_2603_10586_amd as q
    c = case("rand6x7")
    op = q.Operator(c.ctx, c.geom, eps=c.eps, far_prec=PREC_BF16X2, share_transpose=shared)
    th = np.linspace(-30, 30, 4)
    v = q.rhs_plane_waves(c.ctx, c.geom, np.concatenate([th, th]), np.zeros(8), [0] * 4 + [1] * 4)
    x, info, st = op.solve(v, restart=2000, tol=1e-9, max_iter=4000, mode=q.SOLVE_BLOCK_IR)
    assert st == 0 and all(i["converged"] and i["rel_res_true"] <= 1e-9 for i in info)
    assert all(i["n_refine"] >= 2 for i in info)                   # BF16 corrections need refinement
    fac64 = [(r, cc, _c64(Q), _c64(R)) for r, cc, Q, R in _factors(c)]
    ref = _lu_reference(c, fac64, to_host(v))
    xh = to_host(x)
    for r in range(8):
        assert np.linalg.norm(xh[r] - ref[r]) <= 1e-7 * np.linalg.norm(ref[r])
    op.close()


@pytest.mark.parametrize("far_prec", [PREC_C64, PREC_C64_ONLY])
def test_fp32_block_refinement_reaches_its_operator_solution(far_prec):
    """Corrections on FP32 matrix cores (complex64 factors), residuals with the complex128
    factors (C64) or the complex64 ones with FP64 accumulation (C64_ONLY)."""
    import paper_2603_10586_amd as q
    c = case("rand6x7")
    op = q.Operator(c.ctx, c.geom, eps=c.eps, far_prec=far_prec)
    v = q.rhs_plane_waves(c.ctx, c.geom, np.linspace(-20, 20, 6), np.zeros(6), [1] * 6)
    x, info, st = op.solve(v, restart=2000, tol=1e-10, max_iter=4000, mode=q.SOLVE_BLOCK_IR, inner_fp32=True)
    assert st == 0 and all(i["converged"] for i in info)
    fac = _factors(c) if far_prec == PREC_C64 else [(r, cc, _c64(Q), _c64(R)) for r, cc, Q, R in _factors(c)]
    ref = _lu_reference(c, fac, to_host(v))
    xh = to_host(x)
    for r in range(6):
        assert np.linalg.norm(xh[r] - ref[r]) <= 1e-8 * np.linalg.norm(ref[r])
    with pytest.raises(q.QrvieError):                             # complex64 only needs FP32 corrections
        if far_prec == PREC_C64_ONLY:
            op.solve(v, restart=200, tol=1e-8, mode=q.SOLVE_BLOCK_IR)
        else:
            raise q.QrvieError(1, "n/a")
    op.close()
