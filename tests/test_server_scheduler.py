"""Admission, ordering, caching and statistics of the solve server, driven by a fake
executor on the CPU (no GPU): the device work is replaced by timed sleeps."""
import threading
import time
from dataclasses import dataclass

import numpy as np
import pytest

import workloads as W
from paper_2603_10586_amd.server import Server, ServerOpts, replay

GB = 1 << 30


@dataclass
class FakeReq:
    array: object
    incidence: object
    arrival_s: float = 0.0
    tol: float = 1e-6


def req(side, nrhs=1, seed=0, arrival=0.0):
    arr = W.random_lattice(side, seed=seed)
    inc = W.sweep(max(1, (nrhs + 1) // 2))
    inc.theta_deg, inc.phi_deg, inc.pol = inc.theta_deg[:nrhs], inc.phi_deg[:nrhs], inc.pol[:nrhs]
    return FakeReq(arr, inc, arrival)


class Fake:
    """Footprint grows with the particle count; run time with the particle count."""
    lock = threading.Lock()
    running_bytes = 0
    peak_bytes = 0
    builds = 0

    def __init__(self, slot):
        self.slot = slot

    def plan(self, request, opts):
        n = request.array.n_particles
        return ("plan", n), n * GB // 16, n * GB // 8

    def run(self, job, opts, cached):
        with Fake.lock:
            Fake.running_bytes += job.footprint
            Fake.peak_bytes = max(Fake.peak_bytes, Fake.running_bytes)
            if cached is None:
                Fake.builds += 1
        time.sleep(0.002 * job.request.array.n_particles ** 0.5)
        job.x = np.zeros((job.request.incidence.nrhs, 4))
        job.info = [dict(converged=1)] * job.request.incidence.nrhs
        job.status = 0
        with Fake.lock:
            Fake.running_bytes -= job.footprint
        return cached if cached is not None else ("op", job.key)

    def release_cached(self, h):
        pass

    def discard(self, plan):
        pass


@pytest.fixture(autouse=True)
def reset_fake():
    Fake.running_bytes = Fake.peak_bytes = Fake.builds = 0


def test_admission_never_exceeds_the_budget():
    opts = ServerOpts(slots=4, hbm_budget=2 * 64 * GB // 8, op_cache=0)   # two 8x8 requests at a time
    srv = Server(opts, Fake)
    jobs = [srv.result(t) for t in [srv.submit(req(8, seed=s)) for s in range(6)]]
    srv.close()
    assert all(j.status == 0 for j in jobs)
    assert Fake.peak_bytes <= opts.hbm_budget and srv.peak_in_use <= opts.hbm_budget
    assert srv.stats()["requests"] == 6


def test_requests_that_can_never_fit_are_refused():
    srv = Server(ServerOpts(slots=2, hbm_budget=GB, op_cache=0), Fake)
    t = srv.submit(req(12))
    j = srv.result(t)
    srv.close()
    assert j.status == 6 and srv.rejected == 1


def test_small_requests_overtake_a_large_one_that_does_not_fit_yet():
    opts = ServerOpts(slots=3, hbm_budget=(100 + 16) * GB // 8, op_cache=0)
    srv = Server(opts, Fake)
    a = srv.submit(req(10, seed=1))        # 100 particles: fills most of the budget
    b = srv.submit(req(10, seed=2))        # cannot be admitted while a runs
    c = srv.submit(req(4, seed=3))         # 16 particles: fits beside a
    jobs = {t: srv.result(t) for t in (a, b, c)}
    srv.close()
    assert jobs[c].admitted < jobs[b].admitted
    assert all(j.status == 0 for j in jobs.values())


def test_operators_are_reused_for_a_repeated_geometry():
    srv = Server(ServerOpts(slots=1, hbm_budget=64 * GB, op_cache=2), Fake)
    t1 = srv.submit(req(6, seed=7))
    srv.result(t1)
    t2 = srv.submit(req(6, seed=7))        # same geometry
    t3 = srv.submit(req(6, seed=8))
    for t in (t2, t3):
        srv.result(t)
    srv.close()
    assert Fake.builds == 2


def test_poisson_replay_reports_latency_percentiles():
    reqs = W.serving_requests(n=12, seed=3, rate_per_s=200.0, side_lo=3, side_hi=8)
    srv = Server(ServerOpts(slots=3, hbm_budget=64 * GB, op_cache=0), Fake)
    jobs = replay(srv, reqs, time_scale=1.0, timeout=30)
    st = srv.stats()
    srv.close()
    assert st["requests"] == 12 and st["rhs_solves"] == sum(r.incidence.nrhs for r in reqs)
    assert 0 < st["latency_p50_s"] <= st["latency_p99_s"]
    assert all(j.done >= j.admitted >= j.arrival for j in jobs)
