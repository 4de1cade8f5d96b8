"""Cross-approximation compression (compression='aca', the default) against the oracle.

The operator's far blocks are compressed from pivot rows and columns generated on the device
(§6.5: the compression step is a cross approximation after Kurz et al. 2002); no far block
is assembled.  What the method must deliver is unchanged (§5.2, eq. 5.3, read as the relative
Frobenius tolerance per block), so every check here is the sketch path's, with B from the
oracle's ``greens.assemble_block``:

* ||B - Q R||_F <= eps ||B||_F, and the library's certified error agrees with the oracle's;
* Q has orthonormal columns to 1e-12 (R^T for a mirror block);
* the rank is at least the Eckart-Young minimum ``svd_rank`` (blocks of up to 2304 rows);
* the blocks still cover every ordered pair of distinct particles once, and the product
  meets the global bound against the dense Z of a small array;
* without a row cap, blocks of 36,864 rows (256 particles) are compressed and certified:
  the sketch path would have to materialise them.
"""
import numpy as np
import pytest

from oracle import compressed, greens

from gpu_cases import ARRAYS, block_particles, case, ctx, mid, to_dev, to_host

pytestmark = pytest.mark.gpu

EPS = 1e-6
_OPS = {}


def _aca(name, max_block_rows=0, far_prec=0, share_transpose=False):
    """The array's oracle case and its operator built by cross approximation."""
    import paper_2603_10586_amd as q
    c = case(name, max_block_rows=max_block_rows, far_prec=far_prec)
    if not share_transpose:
        return c, c.op
    key = (name, max_block_rows, far_prec)
    if key not in _OPS:
        print(f"[gpu case] shared cross approximation {name} cap={max_block_rows} far_prec={far_prec}", flush=True)
        _OPS[key] = q.Operator(c.ctx, c.geom, eps=EPS, max_block_rows=max_block_rows, far_prec=far_prec,
                               share_transpose=True, compression="aca")
    return c, _OPS[key]


def _certify(disc, order, op, b, eps=EPS, svd_max_rows=2304, slab=None):
    """The oracle's error of exported block b; slab = particles per oracle assembly call
    (large blocks are assembled one row slab at a time)."""
    info, Q, R = op.export_block(b)
    rows, cols = block_particles(order, info)
    if Q is None:
        assert np.linalg.norm(greens.assemble_block(disc, rows, cols)) == 0.0
        return info
    e2 = b2 = 0.0
    step = slab or len(rows)
    for s in range(0, len(rows), step):
        Bs = greens.assemble_block(disc, rows[s:s + step], cols)
        Es = Bs - Q[s * 144:(s + step) * 144] @ R
        e2 += float(np.vdot(Es, Es).real)
        b2 += float(np.vdot(Bs, Bs).real)
        if slab is None and max(Bs.shape) <= svd_max_rows:
            assert Q.shape[1] >= compressed.svd_rank(Bs, eps), info
    err = np.sqrt(e2 / b2)
    assert err <= eps, (info, err)
    assert abs(err - info["rel_err"]) <= 1e-3 * eps, (info, err)
    F = Q if info["row_first"] < info["col_first"] else R.T
    ortho = float(np.max(np.abs(F.conj().T @ F - np.eye(F.shape[1]))))
    assert ortho <= 1e-12, (info, ortho)
    return info


def _stratified(infos, per_level, seed, pick=None):
    rng = np.random.default_rng(seed)
    out = []
    for lvl in sorted({i["level"] for i in infos}):
        idx = [b for b, i in enumerate(infos) if i["level"] == lvl and (pick is None or pick(i))]
        if idx:
            out += list(rng.choice(idx, size=min(per_level, len(idx)), replace=False))
    return out


def test_every_block_of_a_small_array_is_certified_and_the_product_meets_the_bound():
    """rand8x8: every block (direct QR for at most 2 x 2 particles, cross approximation
    above) against the oracle; exact coverage; ||Z_QR x - Z x|| <= eps ||Z_off||_F ||x||."""
    c, op = _aca("rand8x8")
    n = c.array.n_particles
    cover = np.zeros((n, n), dtype=np.int64)
    sizes = set()
    for b in range(op.num_blocks()):
        info = _certify(c.disc, c.order, op, b)
        rows, cols = block_particles(c.order, info)
        cover[np.ix_(rows, cols)] += 1
        sizes.add(info["m"])
    assert np.array_equal(cover, 1 - np.eye(n, dtype=np.int64))
    assert max(sizes) >= 576                                    # blocks of 4 particles took the new path
    rng = np.random.default_rng(18)
    x = rng.standard_normal(c.geom.ndof) + 1j * rng.standard_normal(c.geom.ndof)
    y = to_host(op.apply(to_dev(x)))
    Zoff = c.Z.copy()
    for p in range(n):
        Zoff[p * 144:(p + 1) * 144, p * 144:(p + 1) * 144] = 0
    assert np.linalg.norm(y - c.Z @ x) <= EPS * np.linalg.norm(Zoff) * np.linalg.norm(x)


def test_sampled_blocks_per_level_are_certified():
    """rand16x16: blocks of 576 and 2304 rows on every level, with the rank bound."""
    c, op = _aca("rand16x16")
    infos = [op.export_block(b, factors=False)[0] for b in range(op.num_blocks())]
    seen = set()
    for b in _stratified(infos, 4, seed=21):
        seen.add(_certify(c.disc, c.order, op, int(b))["m"])
    assert {576, 2304} <= seen, seen


def test_blocks_beyond_the_sketch_row_cap_are_certified_without_one():
    """serving33 with no row cap: its far pairs of a 16 x 16 node and an edge node are
    36,864 x 2,304 blocks (and their 2,304 x 36,864 mirrors), compressed without forming them."""
    c, op = _aca("serving33")
    infos = [op.export_block(b, factors=False)[0] for b in range(op.num_blocks())]
    big = [b for b, i in enumerate(infos) if max(i["m"], i["n"]) >= 36864]
    assert big, max(max(i["m"], i["n"]) for i in infos)
    rng = np.random.default_rng(33)
    for b in rng.choice(big, size=min(2, len(big)), replace=False):
        _certify(c.disc, c.order, op, int(b), slab=32)
    for b in _stratified(infos, 2, seed=34, pick=lambda i: max(i["m"], i["n"]) <= 9216):
        _certify(c.disc, c.order, op, int(b))


def test_mid_blocks_are_certified_and_rows_meet_the_operator_bound():
    """Mid-size (32 x 32): sampled blocks of 9216, 2304, 576 and 144 rows certified; sampled
    rows of the product against the oracle's matrix-free rows (as for the sketch path)."""
    m = mid("aca")
    op, infos = m["op"], m["infos"]
    seen = set()
    for b in _stratified(infos, 3, seed=41):
        seen.add(_certify(m["disc"], m["order"], op, int(b), slab=16)["m"])
    assert {9216, 2304, 576, 144} <= seen, seen
    n = m["geom"].ndof
    rng = np.random.default_rng(42)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = to_host(op.apply(to_dev(x)))
    allp = np.arange(m["arr"].n_particles)
    for p in (3, 517, 1020):
        blk = greens.assemble_block(m["disc"], [p], allp)
        zoff = np.sqrt(np.linalg.norm(blk) ** 2 - np.linalg.norm(blk[:, p * 144:(p + 1) * 144]) ** 2)
        diff = np.linalg.norm(y[p * 144:(p + 1) * 144] - blk @ x)
        assert diff <= EPS * zoff * np.linalg.norm(x), (p, diff)
    # the recompressed crosses keep ranks close to the sketch path's (both truncated pivoted QR)
    sk = mid("sketch")["op"].stats()["mean_rank_level"]
    ac = op.stats()["mean_rank_level"]
    for lvl, (a, s) in enumerate(zip(ac, sk)):
        if s > 0:
            assert a <= 1.1 * s + 2.0, (lvl, a, s)


def test_complex64_factors_and_shared_storage_from_crosses():
    """The complex64-only build rounds each chunk's certified factors: exported blocks meet eps
    up to that rounding; a transpose-shared operator's product matches the oracle's."""
    c, op = _aca("rand16x16", far_prec=3, share_transpose=True)
    infos = [op.export_block(b, factors=False)[0] for b in range(op.num_blocks())]
    for b in _stratified(infos, 2, seed=51, pick=lambda i: i["row_first"] < i["col_first"]):
        info, Q, R = op.export_block(int(b))
        rows, cols = block_particles(c.order, info)
        B = greens.assemble_block(c.disc, rows, cols)
        assert np.linalg.norm(B - Q @ R) <= (EPS + 1e-6) * np.linalg.norm(B), info
    rng = np.random.default_rng(52)
    x = rng.standard_normal(c.geom.ndof) + 1j * rng.standard_normal(c.geom.ndof)
    y = to_host(op.apply(to_dev(x)))
    fac = []
    for b in range(op.num_blocks()):
        info, Q, R = op.export_block(b)
        rows, cols = block_particles(c.order, info)
        if Q is not None:
            fac.append((rows, cols, Q, R))
    ref = compressed.compressed_apply(greens.self_blocks(c.disc), fac, x)
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)


def test_footprint_estimate_bounds_the_cross_approximation_build():
    import paper_2603_10586_amd as q
    c = case("tiny")
    geom = q.Geometry(c.ctx, ARRAYS["rand16x16"]())
    chunk = 64 << 20
    est = q.Operator.footprint_estimate(geom, eps=EPS, chunk_bytes=chunk, compression="aca")
    base = c.ctx.bytes_in_use()
    c.ctx.peak_bytes(reset=True)
    op = q.Operator(c.ctx, geom, eps=EPS, chunk_bytes=chunk, compression="aca")
    peak = c.ctx.peak_bytes() - base
    assert op.stats()["device_bytes"] <= est
    assert peak <= est, (peak, est)
    op.close()
    geom.close()


def test_continued_cross_approximations_stay_certified():
    """Starting with 8 crosses, nearly every block uses them all and continues in wider buffers
    (8 -> 16 -> ... from its saved pivots and running estimate); the factors still meet eps
    against the oracle and match the default build's ranks closely."""
    import paper_2603_10586_amd as q
    c = case("rand16x16")
    op = q.Operator(c.ctx, c.geom, eps=EPS, aca_start=8)
    st = op.stats()
    assert st["n_aca_resumed"] >= st["n_aca"] > 0 and st["n_aca_sketch"] == 0
    infos = [op.export_block(b, factors=False)[0] for b in range(op.num_blocks())]
    for b in _stratified(infos, 3, seed=61):
        _certify(c.disc, c.order, op, int(b))
    ref = c.op.stats()["mean_rank_level"]
    for a, r in zip(st["mean_rank_level"], ref):
        assert abs(a - r) <= 0.1 * r + 2.0
    op.close()


def test_uncertified_crosses_are_repeated_then_left_to_the_sketch():
    """A stopping tolerance far above eps (1e4 eps) makes the crosses miss eps: every such block
    is repeated twice with a tenfold tighter tolerance, and the ones still missing go to the
    sketch path; every stored block is certified against the oracle either way."""
    import paper_2603_10586_amd as q
    c = case("rand8x8")
    op = q.Operator(c.ctx, c.geom, eps=EPS, aca_stop=1e4)
    st = op.stats()
    assert st["n_aca_retried"] > 0 and st["n_aca_sketch"] > 0
    for b in range(op.num_blocks()):
        _certify(c.disc, c.order, op, b)
    op.close()


def test_a_second_build_is_bitwise_identical():
    """The build is deterministic: a second cross-approximation build of the mid-size operator
    on the same geometry takes the same steps (ranks, certified errors, continued, repeated and
    fallback counts) and gives the same product bit for bit.  Every reduction has a fixed
    order, and every wave of a cross step holds the pivot before the wave that owns the pivot
    entry normalises it in place."""
    import paper_2603_10586_amd as q
    m = mid("aca")
    op2 = q.Operator(ctx(), m["geom"], eps=EPS, compression="aca")
    s1, s2 = m["op"].stats(), op2.stats()
    for k in ("n_aca", "n_aca_resumed", "n_aca_retried", "n_aca_sketch", "mean_rank_level", "max_block_rel_err"):
        assert s1[k] == s2[k], (k, s1[k], s2[k])
    infos2 = [op2.export_block(b, factors=False)[0] for b in range(op2.num_blocks())]
    assert [(i["rank"], i["rel_err"]) for i in m["infos"]] == [(i["rank"], i["rel_err"]) for i in infos2]
    rng = np.random.default_rng(71)
    n = m["geom"].ndof
    x = to_dev(rng.standard_normal(n) + 1j * rng.standard_normal(n))
    assert np.array_equal(to_host(m["op"].apply(x)), to_host(op2.apply(x)))
    op2.close()
