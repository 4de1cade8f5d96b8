"""Continuous-batching solve server over the C ABI.

Requests (an array of disks plus 1-16 plane-wave right-hand sides and a tolerance)
arrive at any time.  A dispatcher admits queued requests whenever a slot is free and
the sum of the admitted requests' device footprints (operator + Krylov workspaces,
estimated by the library before anything is allocated) stays within the HBM budget;
requests that fit are admitted out of arrival order rather than waiting behind one
that does not (no head-of-line blocking).  Each slot is a worker thread with its own
library context and stream, so admitted requests' kernels overlap on the device.
Operators are compressed once per geometry and kept resident in an LRU cache (their
bytes stay reserved while cached).  Every request's result is independent of what
else runs: the kernels are deterministic and share no mutable state, so a request
gives bitwise the same solution alone and in the mix.

The executor is pluggable: ``DeviceExecutor`` runs requests on the GPU through the
library; tests drive the scheduler with a fake executor on the CPU.
"""
from __future__ import annotations

import collections
import hashlib
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class ServerOpts:
    slots: int = 3                    # requests running concurrently (one stream each)
    hbm_budget: int = 160 << 30       # bytes the admitted requests may hold together
    eps: float = 1e-6                 # compression tolerance of every operator
    restart: int = 3000
    max_iter: int = 3000
    rhs_per_call: int = 8             # right-hand sides advanced together by one solve call
    op_cache: int = 4                 # operators kept resident after their request
    seed: int = 0


@dataclass
class Job:
    ticket: int
    request: object
    arrival: float
    footprint: int = 0
    op_bytes: int = 0
    key: str = ""
    admitted: float | None = None
    started: float | None = None
    done: float | None = None
    x: object = None
    info: list = field(default_factory=list)
    status: int | None = None
    error: str | None = None
    plan: object = None               # executor data carried from admission to the run
    cached: object = None             # resident operator handle reserved at admission

    @property
    def latency(self) -> float:
        return (self.done - self.arrival) if self.done is not None else float("nan")


def geometry_key(array, eps: float, seed: int) -> str:
    h = hashlib.sha256()
    for a in (array.centers, array.radius, array.height, array.eps_r, array.lattice_ij):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(np.float64(eps).tobytes() + np.uint64(seed).tobytes())
    return h.hexdigest()


class Server:
    def __init__(self, opts: ServerOpts, executor_factory, clock=time.perf_counter):
        self.opts = opts
        self.clock = clock
        self._lock = threading.Condition()
        self._queue: collections.OrderedDict[int, Job] = collections.OrderedDict()
        self._ready: collections.deque[Job] = collections.deque()
        self._jobs: dict[int, Job] = {}
        self._next = 0
        self._in_use = 0                     # bytes held by admitted jobs and cached operators
        self._cache: collections.OrderedDict[str, tuple[object, int]] = collections.OrderedDict()
        self._pinned: dict[str, int] = collections.defaultdict(int)   # cache entries in use
        self.peak_in_use = 0
        self.admissions = 0
        self.rejected = 0
        self._closing = False
        self._plan_lock = threading.Lock()
        self.planner = executor_factory(None)
        self._workers = []
        for s in range(opts.slots):
            ex = executor_factory(s)
            t = threading.Thread(target=self._worker, args=(ex,), daemon=True, name=f"qrvie-slot{s}")
            t.start()
            self._workers.append(t)

    # -------------------------------------------------------------- public
    def submit(self, request, arrival: float | None = None) -> int:
        with self._lock:
            t = self._next
            self._next += 1
        job = Job(ticket=t, request=request, arrival=self.clock() if arrival is None else arrival)
        job.key = geometry_key(request.array, self.opts.eps, self.opts.seed)
        with self._plan_lock:
            job.plan, job.op_bytes, job.footprint = self.planner.plan(request, self.opts)
        with self._lock:
            self._jobs[t] = job
            if job.footprint - (job.op_bytes if job.key in self._cache else 0) > self.opts.hbm_budget:
                job.status, job.error, job.done = 6, "request does not fit the HBM budget", self.clock()
                self.rejected += 1
                self.planner.discard(job.plan)
                job.plan = None
                self._lock.notify_all()
                return t
            self._queue[t] = job
            self._admit_locked()
        return t

    def result(self, ticket: int, timeout: float | None = None) -> Job:
        end = None if timeout is None else time.monotonic() + timeout
        with self._lock:
            while self._jobs[ticket].done is None:
                left = None if end is None else end - time.monotonic()
                if left is not None and left <= 0:
                    raise TimeoutError(f"ticket {ticket}")
                self._lock.wait(left)
            return self._jobs[ticket]

    def poll(self, ticket: int) -> bool:
        with self._lock:
            return self._jobs[ticket].done is not None

    def close(self):
        with self._lock:
            self._closing = True
            self._lock.notify_all()
        for t in self._workers:
            t.join()
        for key in list(self._cache):
            self.planner.release_cached(self._cache.pop(key)[0])

    def stats(self) -> dict:
        with self._lock:
            done = [j for j in self._jobs.values() if j.done is not None and j.status in (0, 5)]
        lat = np.array([j.latency for j in done]) if done else np.zeros(1)
        span = (max(j.done for j in done) - min(j.arrival for j in done)) if done else 0.0
        nrhs = sum(len(j.info) for j in done)
        return dict(requests=len(done), rhs_solves=nrhs, rejected=self.rejected, admissions=self.admissions,
                    latency_p50_s=float(np.percentile(lat, 50)), latency_p99_s=float(np.percentile(lat, 99)),
                    makespan_s=span, requests_per_s=len(done) / span if span > 0 else 0.0,
                    rhs_solves_per_s=nrhs / span if span > 0 else 0.0, peak_bytes=self.peak_in_use,
                    queue_wait_p50_s=float(np.percentile([j.admitted - j.arrival for j in done], 50)) if done else 0.0)

    # -------------------------------------------------------------- internals
    def _need(self, job: Job) -> int:
        return job.footprint - (job.op_bytes if job.key in self._cache else 0)

    def _admit_locked(self):
        """Admit queued jobs in arrival order, skipping any that does not fit yet."""
        busy = sum(1 for j in self._jobs.values() if j.admitted is not None and j.done is None)
        for t in list(self._queue):
            if busy >= self.opts.slots:
                break
            job = self._queue[t]
            need = self._need(job)
            while self._in_use + need > self.opts.hbm_budget and self._evict_one_locked():
                pass
            if self._in_use + need <= self.opts.hbm_budget:
                del self._queue[t]
                self._in_use += need
                job.footprint = need
                if job.key in self._cache:
                    self._pinned[job.key] += 1
                    self._cache.move_to_end(job.key)
                    job.cached = self._cache[job.key][0]
                job.admitted = self.clock()
                self.admissions += 1
                busy += 1
                self.peak_in_use = max(self.peak_in_use, self._in_use)
                self._ready.append(job)
                self._lock.notify_all()

    def _evict_one_locked(self) -> bool:
        for key in self._cache:
            if self._pinned[key] == 0:
                handle, nbytes = self._cache.pop(key)
                self._in_use -= nbytes
                self.planner.release_cached(handle)
                return True
        return False

    def _worker(self, ex):
        while True:
            with self._lock:
                while not self._ready and not self._closing:
                    self._lock.wait()
                if not self._ready and self._closing:
                    return
                job = self._ready.popleft()
            job.started = self.clock()
            try:
                new_handle = ex.run(job, self.opts, job.cached)
                err = None
            except Exception as e:       # a failed request frees its slot and reports
                new_handle, err = None, repr(e)
            with self._lock:
                job.done = self.clock()
                if err:
                    job.status, job.error = 4, err
                self._in_use -= job.footprint
                if job.cached is not None:
                    self._pinned[job.key] -= 1
                elif new_handle is not None and self.opts.op_cache > 0 and job.key not in self._cache:
                    # keep the operator resident: its bytes stay reserved
                    self._cache[job.key] = (new_handle, job.op_bytes)
                    self._in_use += job.op_bytes
                    while len(self._cache) > self.opts.op_cache and self._evict_one_locked():
                        pass
                elif new_handle is not None:
                    ex.release_cached(new_handle)
                self._admit_locked()
                self._lock.notify_all()


class DeviceExecutor:
    """Runs requests on the GPU through libqrvie; one instance (context + stream) per slot.

    The planner instance (slot None) creates geometries and asks the library for the
    footprint estimates before anything else is allocated.
    """

    def __init__(self, slot, device: int = 0):
        from . import api
        self.api = api
        self.slot = slot
        self.ctx = api.Context(device)

    def plan(self, request, opts: ServerOpts):
        geom = self.api.Geometry(self.ctx, request.array)
        op_b = self.api.Operator.footprint_estimate(geom, eps=opts.eps)
        nr = min(opts.rhs_per_call, request.incidence.nrhs)
        sol_b = self.api.Operator.solve_footprint_estimate(geom, nr, opts.restart, opts.max_iter)
        return geom, op_b, op_b + sol_b

    def run(self, job: Job, opts: ServerOpts, cached):
        import torch
        req = job.request
        if cached is not None:
            geom, op = cached
            job.plan.close()             # the planned geometry is not needed: the operator is resident
        else:
            geom = job.plan
            op = self.api.Operator(self.ctx, geom, eps=opts.eps, seed=opts.seed)
        inc = req.incidence
        v = self.api.rhs_plane_waves(self.ctx, geom, inc.theta_deg, inc.phi_deg, inc.pol)
        xs, infos, status = [], [], 0
        for r0 in range(0, inc.nrhs, opts.rhs_per_call):
            x, info, st = op.solve(v[r0:r0 + opts.rhs_per_call].contiguous(), restart=opts.restart,
                                   tol=getattr(req, "tol", 1e-6), max_iter=opts.max_iter)
            xs.append(x.cpu())
            infos += info
            status = max(status, st)
        job.x = torch.cat(xs).numpy()
        job.info = infos
        job.status = status
        return (geom, op)

    def release_cached(self, handle):
        geom, op = handle
        op.close()
        geom.close()

    def discard(self, plan):
        if plan is not None:
            plan.close()


def replay(server: Server, requests, time_scale: float = 1.0, timeout: float | None = None) -> list[Job]:
    """Submit requests at their arrival times (seconds x time_scale after the start) and
    wait for all of them; returns the finished jobs in submission order."""
    t0 = server.clock()
    tickets = []
    for req in requests:
        due = t0 + req.arrival_s * time_scale
        while True:
            now = server.clock()
            if now >= due:
                break
            time.sleep(min(due - now, 0.05))
        tickets.append(server.submit(req, arrival=max(due, t0)))
    return [server.result(t, timeout=timeout) for t in tickets]
