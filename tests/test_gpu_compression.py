"""Compression parity at full size: the sketch path (compression='sketch') and the row cap
against the oracle.

Small arrays only reach the direct pivoted-QR path (blocks of at most 2 x 2 particles) and
576-row sketches.  Here the randomised-sketch path that builds every block of 2304 rows or
more (most of the factor bytes at mid-size and beyond) is certified against the oracle's own
re-assembly of each sampled block (§5.2, eq. 5.3, read as the relative Frobenius tolerance
per block):

* ||B - Q R||_F <= eps ||B||_F with B from ``greens.assemble_block`` (and the library's
  certified error agrees with the oracle's);
* Q has orthonormal columns to 1e-12;
* the rank is at least the Eckart-Young minimum ``svd_rank`` (blocks of up to 2304 rows; the
  SVD of a 9216-row block would take minutes on the host).

Operator parity on sampled rows (F2): for a particle p, (Z x)_p from the oracle's
matrix-free rows against the library's (Z_QR x)_p.  Per block the certified bound gives
||((Z_QR - Z) x)_p|| <= sum_b ||E_b||_F ||x_J|| with ||E_b||_F <= eps ||B_b||_F; the test
asserts the row form eps ||Z_off,p||_F ||x||, which is tighter by the share of the blocks'
norm that falls on p's rows and looser by Cauchy-Schwarz (||E_p x|| is about ||E_p||_F ||x|| /
sqrt(n) for a random x, a factor of 384 at mid-size).

The row cap (``max_block_rows``) rewrites the block list (§5.3 grouping: a far pair's child
pairs are again far); a capped operator must still cover every ordered pair of distinct
particles exactly once and certify every block.
"""
import numpy as np
import pytest

from oracle import compressed, greens, grouping

from gpu_cases import ARRAYS, block_particles, case, mid, to_dev, to_host

pytestmark = pytest.mark.gpu

EPS = 1e-6


def _certify(disc, order, op, b, eps=EPS, svd_max_rows=2304):
    info, Q, R = op.export_block(b)
    rows, cols = block_particles(order, info)
    B = greens.assemble_block(disc, rows, cols)
    assert B.shape == (info["m"], info["n"])
    nb = np.linalg.norm(B)
    if Q is None:                                   # rank 0: the whole block is below eps
        assert nb == 0.0
        return info
    err = np.linalg.norm(B - Q @ R) / nb
    assert err <= eps, (info, err)
    assert abs(err - info["rel_err"]) <= 1e-3 * eps, (info, err)
    # the compressed block of a pair (row node first in the internal order) stores an
    # orthonormal Q; its mirror stores the transposed factors, R = Q^T with orthonormal rows
    F = Q if info["row_first"] < info["col_first"] else R.T
    ortho = float(np.max(np.abs(F.conj().T @ F - np.eye(F.shape[1]))))
    assert ortho <= 1e-12, (info, ortho)
    if max(B.shape) <= svd_max_rows:
        assert Q.shape[1] >= compressed.svd_rank(B, eps), info
    return info


def _stratified(infos, per_level, seed, pick=None):
    """Block indices: `per_level` per level (largest blocks of the level first among equals)."""
    rng = np.random.default_rng(seed)
    out = []
    for lvl in sorted({i["level"] for i in infos}):
        idx = [b for b, i in enumerate(infos) if i["level"] == lvl and (pick is None or pick(i))]
        if idx:
            out += list(rng.choice(idx, size=min(per_level, len(idx)), replace=False))
    return out


def test_mid_sketch_blocks_are_certified_against_the_oracle():
    """Mid-size (32 x 32): blocks of 9216, 2304, 576 and 144 rows, sampled on every level."""
    m = mid("sketch")
    levels = {}
    for b in _stratified(m["infos"], 3, seed=1):
        info = _certify(m["disc"], m["order"], m["op"], int(b))
        levels.setdefault(info["m"], 0)
        levels[info["m"]] += 1
    assert {9216, 2304, 576, 144} <= set(levels), levels


def test_mid_product_rows_meet_the_operator_bound_against_the_oracle():
    """F2 on sampled rows: the library's product against the oracle's independent Z."""
    m = mid("sketch")
    n = m["geom"].ndof
    rng = np.random.default_rng(31)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = to_host(m["op"].apply(to_dev(x)))
    allp = np.arange(m["arr"].n_particles)
    for p in (0, 531, 1023):
        blk = greens.assemble_block(m["disc"], [p], allp)          # rows of particle p of Z
        zx = blk @ x
        zoff = np.sqrt(np.linalg.norm(blk) ** 2 - np.linalg.norm(blk[:, p * 144:(p + 1) * 144]) ** 2)
        diff = np.linalg.norm(y[p * 144:(p + 1) * 144] - zx)
        assert diff <= EPS * zoff * np.linalg.norm(x), (p, diff)
        assert diff > 0.0                                          # compressed, not the dense product


def test_serving_array_edge_blocks_are_certified_against_the_oracle():
    """The 33 x 33 serving array with the serving row cap (9216): its 2304 x 144 edge blocks and
    a sample of every level, including split children of capped pairs."""
    c = case("serving33", max_block_rows=9216, compression="sketch")
    assert c.array.n_particles == 1089
    infos = [c.op.export_block(b, factors=False)[0] for b in range(c.op.num_blocks())]
    assert len(infos) == 42714
    assert max(i["m"] for i in infos) <= 9216
    edge = [b for b, i in enumerate(infos) if (i["m"], i["n"]) in ((2304, 144), (144, 2304))]
    assert edge
    picks = list(np.random.default_rng(2).choice(edge, size=4, replace=False)) + _stratified(infos, 2, seed=3)
    for b in picks:
        _certify(c.disc, c.order, c.op, int(b))


def _coverage_from_exports(c):
    n = c.array.n_particles
    cover = np.zeros((n, n), dtype=np.int64)
    for rows, cols, Q, R, info in c.factors():
        cover[np.ix_(rows, cols)] += 1
    return cover


def test_row_cap_keeps_exact_coverage_and_certifies_every_block():
    """rand8x8 with a cap of 288 rows: every 576-row far pair is split into child pairs; the
    exported blocks still cover each ordered pair of distinct particles exactly once, every
    block meets eps against the oracle, and the product meets the global bound against the
    dense Z."""
    c = case("rand8x8", max_block_rows=288, compression="sketch")
    n = c.array.n_particles
    cover = _coverage_from_exports(c)
    assert np.array_equal(cover, 1 - np.eye(n, dtype=np.int64))
    assert max(f[4]["m"] for f in c.factors()) <= 288
    uncapped = grouping.build_blocks(c.array.lattice_ij, c.array.nx, c.array.ny)
    assert len(c.factors()) > len(uncapped)                          # some pairs were split
    for b in range(c.op.num_blocks()):
        _certify(c.disc, c.order, c.op, b)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(c.geom.ndof) + 1j * rng.standard_normal(c.geom.ndof)
    y = to_host(c.op.apply(to_dev(x)))
    Zoff = c.Z.copy()
    for p in range(n):
        Zoff[p * 144:(p + 1) * 144, p * 144:(p + 1) * 144] = 0
    assert np.linalg.norm(y - c.Z @ x) <= EPS * np.linalg.norm(Zoff) * np.linalg.norm(x)


def test_row_cap_splits_sketch_blocks_that_stay_certified():
    """rand16x16 with a cap of 576: 2304-row pairs become 576-row children, compressed on the
    sketch path; a sample per level is certified against the oracle."""
    c = case("rand16x16", max_block_rows=576, compression="sketch")
    infos = [c.op.export_block(b, factors=False)[0] for b in range(c.op.num_blocks())]
    assert max(i["m"] for i in infos) == 576
    for b in _stratified(infos, 3, seed=4):
        _certify(c.disc, c.order, c.op, int(b))


@pytest.mark.parametrize("name,cap,far_prec", [("rand8x8", 288, 0), ("rand6x7", 0, 1), ("rand16x16", 576, 0)])
def test_footprint_estimate_bounds_the_sketch_build(name, cap, far_prec):
    """The estimate covers the built operator and the build's peak (transient buffers
    included), following the same capped block list."""
    import paper_2603_10586_amd as q
    c = case("tiny")
    arr = ARRAYS[name]()
    geom = q.Geometry(c.ctx, arr)
    chunk = 64 << 20
    est = q.Operator.footprint_estimate(geom, eps=EPS, max_block_rows=cap, far_prec=far_prec, chunk_bytes=chunk,
                                        compression="sketch")
    base = c.ctx.bytes_in_use()
    c.ctx.peak_bytes(reset=True)
    op = q.Operator(c.ctx, geom, eps=EPS, max_block_rows=cap, far_prec=far_prec, chunk_bytes=chunk,
                    compression="sketch")
    peak = c.ctx.peak_bytes() - base
    assert op.stats()["device_bytes"] <= est
    assert peak <= est, (peak, est)
    op.close()
    geom.close()


@pytest.mark.parametrize("compression", ["sketch", "aca"])
def test_matrix_core_products_over_edge_blocks_match_the_oracle(compression):
    """The 33 x 33 serving array (row cap 9216) has 2304 x 144 edge blocks, the shape on which
    an FP64-MFMA variant of the build GEMM once failed certification.  Its factors were built
    by CGS2 panels on FP64 matrix cores (certified above); here the block product (16 and 20
    right-hand sides: FP64-MFMA strip kernels over every Q and R panel, edge strips included)
    must match the oracle's product of the exported factors."""
    c = case("serving33", max_block_rows=9216, compression=compression)
    fac = [(r, cc, Q, R) for r, cc, Q, R, _ in c.factors()]
    edge = [i for *_, i in c.factors() if (i["m"], i["n"]) in ((2304, 144), (144, 2304))]
    assert edge
    sb = greens.self_blocks(c.disc)
    rng = np.random.default_rng(90)
    for nrhs in (16, 20):
        x = rng.standard_normal((nrhs, c.geom.ndof)) + 1j * rng.standard_normal((nrhs, c.geom.ndof))
        y = to_host(c.op.apply(to_dev(x)))
        ref = compressed.compressed_apply(sb, fac, x.T).T
        for r in range(nrhs):
            assert np.linalg.norm(y[r] - ref[r]) <= 1e-12 * np.linalg.norm(ref[r]), (nrhs, r)
