"""Continuous-batching solve server: a binding of the library's native server
(qrvie_server_* in include/qrvie.h; argument marshalling only).

Requests (an array of disks, 1-64 plane-wave right-hand sides and a tolerance) are
submitted at any time.  The library admits them by device footprint without head-of-line
blocking, runs admitted requests concurrently (one worker and stream per slot), compresses
each geometry once and keeps its operator resident (LRU), and reports latency percentiles
and throughput.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L
from .api import QrvieError, _dptr, array_desc


@dataclass
class ServerOpts:
    slots: int = 3                    # requests running concurrently (one worker + stream each)
    hbm_budget: int = 160 << 30       # bytes the admitted requests and cached operators may hold
    eps: float = 1e-6                 # compression tolerance of every operator
    restart: int = 3000               # basis vectors per cycle
    max_iter: int = 3000
    mode: int = L.SOLVE_BLOCK         # every request's right-hand sides share one block Krylov space
    block_width: int = 0
    op_cache: int = 4                 # operators kept resident after their request
    seed: int = 0
    tune_tiles: bool = True           # autotune each new operator's block product tiles
    max_bypass: int = 6               # later admissions that may overtake a waiting request


@dataclass
class Result:
    ticket: int
    status: int
    x: np.ndarray                     # (nrhs, n) complex128, caller order
    info: list = field(default_factory=list)
    arrival: float = 0.0              # server clock, seconds
    admitted: float = 0.0
    done: float = 0.0

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Server:
    def __init__(self, opts: ServerOpts = ServerOpts(), device: int = 0):
        self.lib = L.load()
        self.opts = opts
        o = L.ServerOptsC(slots=opts.slots, hbm_budget=opts.hbm_budget, eps=opts.eps, restart=opts.restart,
                          max_iter=opts.max_iter, mode=opts.mode, block_width=opts.block_width,
                          op_cache=opts.op_cache, seed=opts.seed, tune_tiles=1 if opts.tune_tiles else 0,
                          max_bypass=opts.max_bypass)
        h = C.c_void_p()
        st = self.lib.qrvie_server_create(device, C.byref(o), C.byref(h))
        if st != L.OK:
            raise QrvieError(st, "server_create: invalid options or device")
        self.h = h
        self._n = {}

    def _check(self, st: int, what: str):
        if st not in (L.OK, L.NOT_CONVERGED):
            raise QrvieError(st, f"{what}: {self.lib.qrvie_server_last_error(self.h).decode()}")
        return st

    def submit(self, request) -> int:
        """request: .array, .incidence (theta_deg, phi_deg, pol) and optionally .tol."""
        d, keep = array_desc(request.array)
        inc = request.incidence
        th = np.ascontiguousarray(inc.theta_deg, dtype=np.float64)
        ph = np.ascontiguousarray(inc.phi_deg, dtype=np.float64)
        po = np.ascontiguousarray(inc.pol, dtype=np.int32)
        t = C.c_uint64()
        self._check(self.lib.qrvie_server_submit(self.h, C.byref(d), int(th.size), _dptr(th, C.c_double),
                                                 _dptr(ph, C.c_double), _dptr(po, C.c_int32),
                                                 float(getattr(request, "tol", 1e-6)), C.byref(t)), "submit")
        self._n[t.value] = (d.n * 144, int(th.size))
        return t.value

    def poll(self, ticket: int) -> bool:
        done = C.c_int32()
        self._check(self.lib.qrvie_server_poll(self.h, ticket, C.byref(done)), "poll")
        return bool(done.value)

    def result(self, ticket: int, timeout: float | None = None) -> Result:
        done = C.c_int32()
        self._check(self.lib.qrvie_server_wait(self.h, ticket, -1.0 if timeout is None else float(timeout),
                                               C.byref(done)), "wait")
        if not done.value:
            raise TimeoutError(f"ticket {ticket}")
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        self._check(self.lib.qrvie_server_request_times(self.h, ticket, C.byref(a), C.byref(b), C.byref(c)), "times")
        n, nrhs = self._n.pop(ticket)
        x = np.zeros((nrhs, n), dtype=np.complex128)
        infos = (L.SolveInfo * nrhs)()
        st = self.lib.qrvie_server_fetch(self.h, ticket, C.c_void_p(x.ctypes.data), n, infos)
        info = [{f: getattr(i, f) for f, _ in L.SolveInfo._fields_} for i in infos]
        return Result(ticket, st, x, info, a.value, b.value, c.value)

    def last_error(self) -> str:
        """The server's most recent error message (a failed request or call)."""
        return self.lib.qrvie_server_last_error(self.h).decode()

    def stats(self) -> dict:
        s = L.ServerStatsC()
        self._check(self.lib.qrvie_server_get_stats(self.h, C.byref(s)), "stats")
        return {f: getattr(s, f) for f, _ in L.ServerStatsC._fields_}

    def close(self):
        if getattr(self, "h", None):
            self.lib.qrvie_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server: Server, requests, time_scale: float = 1.0, timeout: float | None = None,
           report=None) -> list[Result]:
    """Submit requests at their arrival times (seconds x time_scale after the start) and wait
    for all of them; returns the results in submission order.  `report(text)`, if given, is
    called for every submission and every finished request."""
    t0 = time.perf_counter()
    tickets, results = [], {}

    def collect():
        for t in tickets:
            if t not in results and server.poll(t):
                results[t] = server.result(t)
                if report:
                    r = results[t]
                    report(f"finished ticket {t}: status {r.status}, latency {r.latency:.2f} s, "
                           f"{len(results)}/{len(requests)} done"
                           + (f" ({server.last_error()})" if r.status not in (0, 5) else ""))

    for req in requests:
        due = t0 + req.arrival_s * time_scale
        while time.perf_counter() < due:
            collect()
            time.sleep(min(max(due - time.perf_counter(), 0.0), 0.05))
        tickets.append(server.submit(req))
        if report:
            report(f"submitted request {len(tickets)}/{len(requests)} ({req.array.n_particles} particles, "
                   f"{len(req.incidence.theta_deg)} waves)")
    while len(results) < len(tickets):
        collect()
        time.sleep(0.05)
    return [results[t] for t in tickets]
