"""The paper's test geometry on the GPU against the oracle: Vogel spirals of voxelised gold
spheres (§6.1) grouped on the paper's grid (§5.3, §5.4), compressed by cross approximation
and solved by unrestarted GMRES to 1e-4 (the paper's solver setting, §6).

* the library's grid (finest-level block of every particle, number of levels) and block list
  equal the oracle's ``grouping.paper_grid`` / ``build_blocks_paper`` exactly (integers);
* cell centres and volumes equal the oracle's ``sphere_cells`` placement;
* sampled blocks per level meet ||B - Q R||_F <= eps ||B||_F against ``greens.assemble_block``;
* the solve's true residual against the oracle's independent Z (matrix-free, every row)
  is within tol ||v|| plus the operator error eps ||Z_off||_F ||x||.
"""
import numpy as np
import pytest

import workloads as W
from oracle import discretise, greens, grouping

from gpu_cases import block_particles, ctx, to_host

pytestmark = pytest.mark.gpu

EPS = 1e-6
_V = {}


def vogel(n):
    import paper_2603_10586_amd as q
    if n not in _V:
        print(f"[gpu case] vogel {n}: geometry and cross-approximation operator", flush=True)
        arr = W.vogel(n)
        geom = q.Geometry(ctx(), arr)
        op = q.Operator(ctx(), geom, eps=EPS)
        _V[n] = dict(arr=arr, geom=geom, op=op, order=geom.order(), disc=discretise.Discretisation(arr))
    return _V[n]


@pytest.mark.parametrize("n", [100, 500])
def test_grid_and_blocks_match_the_oracle(n):
    v = vogel(n)
    L, ij, _, _ = grouping.paper_grid(v["arr"].centers)
    assert v["geom"].n_levels == L
    assert np.array_equal(v["geom"].blocks(), ij)
    ref = {(b.level, b.rows, b.cols) for b in grouping.build_blocks_paper(v["arr"].centers)[0]}
    got = set()
    for b in range(v["op"].num_blocks()):
        info = v["op"].export_block(b, factors=False)[0]
        rows, cols = block_particles(v["order"], info)
        got.add((info["level"], tuple(sorted(rows.tolist())), tuple(sorted(cols.tolist()))))
    assert got == ref


def test_sphere_cells_match_the_oracle():
    v = vogel(100)
    c, vol = v["geom"].cells()
    assert np.allclose(c.reshape(100, 48, 3), v["disc"].pos, rtol=0, atol=1e-14)
    assert np.allclose(vol.reshape(100, 48), v["disc"].vol[:, None], rtol=1e-15, atol=0)


def test_sampled_blocks_are_certified_against_the_oracle():
    v = vogel(500)
    infos = [v["op"].export_block(b, factors=False)[0] for b in range(v["op"].num_blocks())]
    rng = np.random.default_rng(5)
    seen = set()
    for lvl in sorted({i["level"] for i in infos}):
        idx = [b for b, i in enumerate(infos) if i["level"] == lvl]
        big = max(idx, key=lambda b: infos[b]["m"] * infos[b]["n"])        # the largest of the level
        for b in {big, *rng.choice(idx, size=min(2, len(idx)), replace=False)}:
            info, Q, R = v["op"].export_block(int(b))
            rows, cols = block_particles(v["order"], info)
            B = greens.assemble_block(v["disc"], rows, cols)
            err = np.linalg.norm(B - Q @ R) / np.linalg.norm(B)
            assert err <= EPS, (info, err)
            assert abs(err - info["rel_err"]) <= 1e-3 * EPS
            seen.add(lvl)
    assert 1 in seen                                                      # the 3 x 3 level compresses


def test_unrestarted_gmres_meets_the_paper_tolerance_against_the_oracle():
    """One normally incident x-polarised plane wave, GMRES without restart (at most 5000
    iterations) to 1e-4, the preconditioner of §4; the stage counters of the paper's table
    are filled (products, preconditioner applications, their times and the Krylov time)."""
    import paper_2603_10586_amd as q
    v = vogel(100)
    rhs = q.rhs_plane_waves(ctx(), v["geom"], [0.0], [0.0], [1])
    x, info, st = v["op"].solve(rhs, restart=5000, max_iter=5000, tol=1e-4)
    i = info[0]
    print(f"[vogel 100] {i['iterations']} iterations, products {i['n_apply']}, true residual {i['rel_res_true']:.2e}",
          flush=True)
    assert st == 0 and i["converged"] and i["restarts"] == 0
    assert i["n_apply"] >= i["iterations"] and i["n_prec"] >= i["iterations"]
    assert i["t_apply_s"] > 0 and i["t_krylov_s"] > 0 and i["t_total_s"] >= i["t_apply_s"]
    vh, xh = to_host(rhs)[0], to_host(x)[0]
    # caller-order solution against the oracle's matrix-free Z (every row)
    zx = greens.matvec_free(v["disc"], xh)
    Zoff2 = 0.0
    allp = np.arange(100)
    for p in range(100):
        blk = greens.assemble_block(v["disc"], [p], allp)
        Zoff2 += np.linalg.norm(blk) ** 2 - np.linalg.norm(blk[:, p * 144:(p + 1) * 144]) ** 2
    assert np.linalg.norm(vh - zx) <= 1e-4 * np.linalg.norm(vh) + EPS * np.sqrt(Zoff2) * np.linalg.norm(xh)
    # the oracle's right-hand side is the library's
    ref = greens.plane_wave_rhs(v["disc"], [0.0], [0.0], [1])
    assert np.allclose(vh, np.asarray(ref).reshape(-1), rtol=0, atol=1e-12 * np.abs(vh).max())
