"""Continuous-batching server on the GPU: results are the same alone and in the mix."""
import numpy as np
import pytest

import workloads as W
from oracle import compressed, discretise, greens

pytestmark = pytest.mark.gpu


def _requests():
    rng = np.random.default_rng(11)
    out = []
    for rid, side in enumerate([3, 5, 4, 6, 3]):
        arr = W.random_lattice(side, seed=100 + rid)
        inc = W.random_incidence(int(rng.integers(1, 4)), rng)
        out.append(W.Request(rid=rid, arrival_s=0.0, array=arr, incidence=inc, tol=1e-8))
    return out


def test_results_are_bitwise_identical_alone_and_in_the_mix():
    from paper_2603_10586_amd.server import DeviceExecutor, Server, ServerOpts
    reqs = _requests()
    opts = dict(hbm_budget=8 << 30, restart=400, max_iter=2000, op_cache=0)
    alone_srv = Server(ServerOpts(slots=1, **opts), DeviceExecutor)
    alone = [alone_srv.result(alone_srv.submit(r), timeout=120) for r in reqs]
    alone_srv.close()
    mix_srv = Server(ServerOpts(slots=3, **opts), DeviceExecutor)
    tickets = [mix_srv.submit(r) for r in reqs]
    mix = [mix_srv.result(t, timeout=120) for t in tickets]
    st = mix_srv.stats()
    mix_srv.close()
    for a, b in zip(alone, mix):
        assert a.status == 0 and b.status == 0, (a.error, b.error)
        assert np.array_equal(a.x, b.x)
        assert all(i["converged"] and i["rel_res_true"] <= 1e-8 for i in b.info)
    assert st["requests"] == len(reqs) and st["peak_bytes"] <= 8 << 30
    # requests overlapped: more than one was admitted before the first finished
    first_done = min(j.done for j in mix)
    assert sum(j.admitted < first_done for j in mix) >= 2


def test_served_solution_matches_the_oracle_on_the_same_operator():
    import paper_2603_10586_amd as q
    from paper_2603_10586_amd.server import DeviceExecutor, Server, ServerOpts
    r = _requests()[1]
    srv = Server(ServerOpts(slots=1, hbm_budget=8 << 30, restart=400, max_iter=2000, op_cache=1), DeviceExecutor)
    job = srv.result(srv.submit(r), timeout=120)
    geom, op = srv._cache[job.key][0]
    order = geom.order()
    fac = []
    for b in range(op.num_blocks()):
        bi, Q, R = op.export_block(b)
        rows = order[bi["row_first"]:bi["row_first"] + bi["row_count"]]
        cols = order[bi["col_first"]:bi["col_first"] + bi["col_count"]]
        fac.append((rows, cols, Q, R))
    srv.close()
    disc = discretise.Discretisation(r.array)
    ZQR = compressed.dense_from_factors(greens.self_blocks(disc), fac)
    v = greens.plane_wave_rhs(disc, r.incidence.theta_deg, r.incidence.phi_deg, r.incidence.pol)
    ref = np.linalg.solve(ZQR, v).T
    for k in range(r.incidence.nrhs):
        assert np.linalg.norm(job.x[k] - ref[k]) <= 1e-6 * np.linalg.norm(ref[k])
