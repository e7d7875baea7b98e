"""Serving loop: flow-past-particle solves admitted into one resident batch.

Requests (a lattice, its solids and its boundary method) arrive over time.  A
request is admitted as soon as the batch has a free slot and a free pool
range of the request's footprint (``lbm_workspace_bytes``: populations, flags,
links, Lagrangian data, history, with link and point capacities sized to the
request's solids); its lattice then stays resident and is
advanced together with every other admitted lattice by the batch (continuous
batching: members join and leave between check intervals while the others
keep running).  Every ``check_every`` steps one device launch measures, per
member, the relative force change over the interval; a member whose change is
below ``tol`` (or that reached ``step_cap``) is read out and released.

Latency is split into queueing (arrival -> admission) and service (admission
-> result).  All computation runs in liblbm.so; this module only orders calls.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque
from typing import Callable, Iterable, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    """One solve: a workloads.Case plus its arrival time (seconds from start)."""

    rid: int
    arrival: float
    case: object
    n_iter: int = 5
    footprint: int = 0
    admitted: Optional[float] = None
    finished: Optional[float] = None
    steps: int = 0
    converged: bool = False
    capped: bool = False
    diverged: bool = False
    rejected: bool = False
    force: Optional[np.ndarray] = None  # [nsolid, 6] at the last step
    change: float = -1.0

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival

    @property
    def queue_time(self):
        return None if self.admitted is None else self.admitted - self.arrival

    @property
    def service_time(self):
        return None if self.finished is None or self.admitted is None else self.finished - self.admitted


def capacities(case):
    """(max_links, max_lagrangian) that a request's solids need, or 0 for the
    library's bound from the lattice size where no bound is known here.

    A bounce-back sphere of radius R (D3Q19) has, for each direction e_i, one
    link on every lattice line along e_i that holds a solid node (the first
    fluid node past the solid run: the sphere is convex), so at most as many
    as such lines pass within R of the centre.  Those lines cross the plane
    normal to e_i in a 2-D lattice of |e_i| points per unit area whose
    Voronoi cells lie within rho_i of their point (rho = sqrt(2)/2 for the
    6 axis directions, sqrt(3/2)/2 for the 12 diagonal ones), which bounds
    their number by |e_i| pi (R + rho_i)^2.  Such a request reserves no IBM
    space (-1).  IBM requests keep the library's bounds: the point capacity
    also sizes the table of the summed direct-forcing iterations, which a
    tighter capacity could leave out (the iterations would then run one by
    one)."""
    if case.lattice != "D3Q19" or case.method == "IBM" or \
            any(s["kind"] != "sphere" or s["inverted"] for s in case.solids):
        return 0, 0
    ra, rd = math.sqrt(2.0) / 2.0, math.sqrt(1.5) / 2.0
    links = sum(6.0 * math.pi * (s["radius"] + ra) ** 2 + 12.0 * math.sqrt(2.0) * math.pi * (s["radius"] + rd) ** 2
                for s in case.solids)
    return int(links) + 64, -1


def footprint(lbm, case, storage=None) -> int:
    """Device bytes a request takes in the pool (its context workspace)."""
    max_links, max_lagrangian = capacities(case)
    return lbm.Batch.footprint(case.lattice, case.collision, storage or case.storage, case.shape, case.tau,
                               max_solids=max(1, len(case.solids)), max_links=max_links,
                               max_lagrangian=max_lagrangian)


def initial_velocity(case):
    """Uniform start velocity of a solve (meta["U_init"] along its body force), or None (from rest)."""
    U0 = case.meta.get("U_init")
    gn = np.asarray(case.g, dtype=np.float64)
    if not U0 or not np.any(gn):
        return None
    return tuple(U0 * gn / np.linalg.norm(gn))


def outcome(change, time, step_cap, tol, nsolid):
    """What a check does with a running request: "converged" (relative force
    change below tol), "diverged" (the change is not a number: the member's
    force, hence its populations, went non-finite), "capped" (step cap
    reached, or no solid to converge), or None (keep running)."""
    if change != change:  # NaN
        return "diverged"
    if 0.0 <= change < tol:
        return "converged"
    if time >= step_cap or not nsolid:
        return "capped"
    return None


def percentile(values, q):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty sequence; None if empty."""
    v = sorted(values)
    if not v:
        return None
    k = max(1, int(np.ceil(q / 100.0 * len(v))))
    return float(v[min(k, len(v)) - 1])


class Admission:
    """First-fit admission in arrival order: the oldest waiting request that
    fits is admitted first; a request too large for the current free memory
    does not block smaller ones behind it.  ``try_admit(req)`` returns a
    handle or None (no slot / no contiguous range)."""

    def __init__(self, try_admit: Callable[[Request], object]):
        self.try_admit = try_admit
        self.queue: deque = deque()

    def push(self, req: Request):
        self.queue.append(req)

    def admit_all(self, now: float) -> List[tuple]:
        out = []
        keep = deque()
        while self.queue:
            req = self.queue.popleft()
            h = self.try_admit(req)
            if h is None:
                keep.append(req)
            else:
                req.admitted = now
                out.append((req, h))
        self.queue = keep
        return out


class Server:
    """A batch of resident lattices serving a request trace."""

    def __init__(self, pool_bytes: int, max_slots: int = 128, storage: str = "F32", check_every: int = 100,
                 tol: float = 1e-6, step_cap: int = 200000, clock=time.perf_counter, warm_start: bool = True):
        from . import lbm

        self.lbm = lbm
        self.storage = storage
        self.batch = lbm.Batch("D3Q19", storage, max_slots=max_slots, pool_bytes=pool_bytes)
        self.pool_bytes = pool_bytes
        self.check_every = int(check_every)
        self.tol = float(tol)
        self.step_cap = int(step_cap)
        self.clock = clock
        # start each solve from the uniform flow its case estimates (meta["U_init"], along the
        # body force) instead of from rest: the same steady state, a shorter transient
        self.warm_start = bool(warm_start)
        self.active = {}  # Member -> Request
        self.cell_steps = 0

    def _try_admit(self, req: Request):
        c = req.case
        if req.footprint > self.pool_bytes:
            req.rejected = True
            return None
        max_links, max_lagrangian = capacities(c)
        m = self.batch.admit(c.collision, self.storage, c.shape, c.tau, g=c.g,
                             max_solids=max(1, len(c.solids)), max_links=max_links,
                             max_lagrangian=max_lagrangian)
        if m is None:
            return None
        m.set_solids(c.solids, c.method, n_iter=req.n_iter)
        u0 = initial_velocity(c) if self.warm_start else None
        if u0 is not None:
            m.set_equilibrium(1.0, u0)
        return m

    def _finish(self, m, req, now):
        req.finished = now
        req.steps = m.time
        req.force = m.force_torque() if m.nsolid else None
        self.batch.release(m)
        del self.active[m]

    def run(self, requests: Iterable[Request], wall_limit: Optional[float] = None, log=None,
            stop_after: Optional[int] = None):
        """Serve the requests (sorted by arrival) until all are done, wall_limit
        seconds have passed or stop_after requests have completed; returns the
        summary dict of ``stats``."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        for r in reqs:
            r.footprint = footprint(self.lbm, r.case, self.storage)
        pending = deque(reqs)
        adm = Admission(self._try_admit)
        t0 = self.clock()
        now = 0.0
        next_note = 20.0
        while True:
            now = self.clock() - t0
            if log and now >= next_note:  # a status line from the loop every 20 s
                log(f"serving: {now:.0f} s, {sum(1 for r in reqs if r.finished is not None)} done, "
                    f"{len(self.active)} running, {len(adm.queue)} queued")
                next_note += 20.0
            while pending and pending[0].arrival <= now:
                adm.push(pending.popleft())
            for req, m in adm.admit_all(now):
                self.active[m] = req
            adm.queue = deque(r for r in adm.queue if not r.rejected)
            if wall_limit is not None and now >= wall_limit:
                break
            if stop_after is not None and sum(1 for r in reqs if r.finished is not None) >= stop_after:
                break
            if not self.active:
                if not pending and not adm.queue:
                    break
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival - now, 0.05)))
                    continue
                # nothing running and the head of the queue never fits: reject it
                adm.queue[0].rejected = True
                adm.queue.popleft()
                continue
            cells = sum(m.N for m in self.active)
            self.batch.step(self.check_every)
            self.cell_steps += cells * self.check_every
            change = self.batch.force_change(self.check_every)
            now = self.clock() - t0
            for m, req in list(self.active.items()):
                ch = change.get(m, -1.0)
                req.change = ch
                end = outcome(ch, m.time, self.step_cap, self.tol, m.nsolid)
                if end is not None:
                    req.converged = end == "converged"
                    req.capped = end == "capped"
                    req.diverged = end == "diverged"
                    self._finish(m, req, now)
                    if log:
                        log(f"req {req.rid}: {end} after {req.steps} steps, latency {req.latency:.3f} s")
        wall = self.clock() - t0
        for m, req in self.active.items():
            req.steps = m.time
        return stats(reqs, wall, self.cell_steps, in_flight=list(self.active.values()), queued=len(adm.queue))

    def close(self):
        for m in list(self.active):
            self.batch.release(m)
        self.active.clear()
        self.batch.close()


def stats(reqs, wall, cell_steps=0, in_flight=(), queued=0):
    """Summary of a serving run; in_flight: the requests still running at the end."""
    done = [r for r in reqs if r.finished is not None]
    running = list(in_flight)
    conv = [r for r in done if r.converged]
    lat = [r.latency for r in done]
    return {
        "offered": len(reqs),
        "arrived_by_end": sum(1 for r in reqs if r.arrival <= wall),
        "completed": len(done),
        "converged": len(conv),
        "capped": sum(1 for r in done if r.capped),
        "diverged": sum(1 for r in done if r.diverged),
        "rejected": sum(1 for r in reqs if r.rejected),
        "in_flight_at_end": len(running),
        "in_flight_mean_steps": float(np.mean([r.steps for r in running])) if running else None,
        "in_flight_median_change": (float(np.median([r.change for r in running if r.change >= 0]))
                                    if any(r.change >= 0 for r in running) else None),
        "queued_at_end": queued,
        "wall_s": wall,
        "solves_per_s": len(done) / wall if wall > 0 else 0.0,
        "latency_n": len(lat),
        "latency_p50_s": percentile(lat, 50),
        "latency_p99_s": percentile(lat, 99),
        "queue_p50_s": percentile([r.queue_time for r in done], 50),
        "queue_p99_s": percentile([r.queue_time for r in done], 99),
        "service_p50_s": percentile([r.service_time for r in done], 50),
        "service_p99_s": percentile([r.service_time for r in done], 99),
        "mean_steps": float(np.mean([r.steps for r in done])) if done else None,
        "mlups": cell_steps / wall / 1e6 if wall > 0 else 0.0,
    }


def requests_from_trace(trace, n_iter=5):
    """Requests from workloads.request_trace entries."""
    return [Request(k, e["arrival"], e["case"], n_iter=n_iter) for k, e in enumerate(trace)]
