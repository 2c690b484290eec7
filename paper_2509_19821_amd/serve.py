"""Continuous-batching solve server over a pool of resident GMPEA instances.

Requests (a CMOP, method parameters and a deadline) arrive over time. A request
is admitted into the pool as soon as its device-memory footprint fits the
budget; until then it waits in arrival order. Every loop iteration advances all
resident solves by a few batched generations (one launch per phase for all of
them, per generation): as many as are expected to fit before the earliest
deadline among them, at most max_chunk, at least one. When a solve's deadline
has passed, the loop stops it at that generation boundary, as in the paper's fixed-time protocol (a run reaching its
time limit outputs its current set), takes its feasible non-dominated front
(population 1) and frees its slot for waiting requests.

Each delivered result records how many generations the solve received, so it
can be reproduced exactly: an instance advanced alone for that many generations
computes the same front bit for bit. A request that carries a reference front
(and optionally an HV reference point) also gets the front's IGD (Eq. (14))
and Monte Carlo HV (Eq. (15)) at its deadline, computed on the device before
the slot is freed.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from .gmpea import Pool


@dataclass
class Request:
    rid: int
    problem: dict
    config: dict
    deadline_s: float          # time allowed after arrival
    arrival: float = 0.0       # wall-clock arrival (seconds since the server started)
    reference: np.ndarray | None = field(default=None, repr=False)  # IGD reference front (k x m)
    hv_point: np.ndarray | None = field(default=None, repr=False)   # HV reference point (m)


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    delivered: float
    deadline: float            # absolute deadline (arrival + deadline_s)
    generations: int
    n: int
    front_f: np.ndarray = field(repr=False)
    front_x: np.ndarray = field(repr=False)
    igd: float | None = None   # at the deadline, on the device (requests with a reference front)
    hv: float | None = None

    @property
    def latency(self):
        return self.delivered - self.arrival

    @property
    def lateness(self):
        return self.delivered - self.deadline


class Server:
    """Single-threaded serving loop on one GPU (one pool, one stream)."""

    def __init__(self, budget_bytes: int, clock=time.perf_counter, keep_fronts: bool = True,
                 hv_samples: int = 1 << 18, max_chunk: int = 8, pool=None):
        # pool: any object with Pool's try_admit / instance / step / sync /
        # release / close (the scheduling is tested on the host with a stand-in)
        self.pool = pool if pool is not None else Pool(budget_bytes)
        self.clock = clock
        self.t0 = None
        self.waiting = collections.deque()
        self.active = {}       # slot -> (request, admitted time, start generation)
        self.results = []
        self.offspring = 0     # offspring evaluated and selected so far
        self.steps = 0
        self.keep_fronts = keep_fronts
        self.hv_samples = hv_samples
        self.max_chunk = max(1, int(max_chunk))
        self.gen_s = None      # running estimate of one batched generation's duration
        self.host_s = {"admit": 0.0, "step": 0.0, "harvest": 0.0}  # wall time per activity

    def now(self) -> float:
        if self.t0 is None:
            self.t0 = self.clock()
        return self.clock() - self.t0

    def submit(self, req: Request):
        self.waiting.append(req)

    def _admit(self):
        while self.waiting:
            req = self.waiting[0]
            slot = self.pool.try_admit(req.problem, req.config)
            if slot is None:
                if not self.active:
                    raise MemoryError("request %d does not fit an empty pool" % req.rid)
                return  # wait for a slot to free up
            self.waiting.popleft()
            inst = self.pool.instance(slot)
            self.active[slot] = (req, self.now(), inst.n)

    def _harvest(self, force: bool = False):
        t = self.now()
        for slot in list(self.active):
            req, admitted, n = self.active[slot]
            if force or t >= req.arrival + req.deadline_s:
                inst = self.pool.instance(slot)
                fr = inst.front(with_x=self.keep_fronts)
                gens = int(inst.read("GEN")[0])
                delivered = self.now()
                q = {"igd": None, "hv": None}
                if req.reference is not None or req.hv_point is not None:
                    q = inst.quality(req.reference, req.hv_point, hv_samples=self.hv_samples)
                self.results.append(Result(req.rid, req.arrival, admitted, delivered,
                                           req.arrival + req.deadline_s, gens, n,
                                           fr["f"] if self.keep_fronts else fr["f"][:0],
                                           fr["x"],
                                           q["igd"], q["hv"]))
                self.pool.release(slot)
                del self.active[slot]

    def _chunk(self) -> int:
        """Generations for this step: those expected to end before the earliest
        resident deadline (one generation's duration estimated from the last
        steps), within [1, max_chunk]."""
        if self.gen_s is None or self.max_chunk == 1:
            return 1
        now = self.now()
        left = min(req.arrival + req.deadline_s for (req, _, _) in self.active.values()) - now
        return int(min(self.max_chunk, max(1, left // self.gen_s)))

    def step(self):
        """Advance every resident solve by one or more generations, admit what
        fits while the GPU works (new solves join from the next step on), then
        deliver the solves whose deadline has passed."""
        c = self.clock
        t0 = c()
        stepped = bool(self.active)
        k = 0
        if stepped:
            k = self._chunk()
            self.pool.step(k)
            self.steps += k
            self.offspring += k * sum(2 * n for (_, _, n) in self.active.values())
        t1 = c()
        self._admit()
        t2 = c()
        if stepped:
            self.pool.sync()
        t3 = c()
        if stepped:  # per generation, admission included: what a step really costs
            per = (t3 - t0) / k
            self.gen_s = per if self.gen_s is None else 0.8 * self.gen_s + 0.2 * per
        self._harvest()
        t4 = c()
        self.host_s["step"] += (t1 - t0) + (t3 - t2)
        self.host_s["admit"] += t2 - t1
        self.host_s["harvest"] += t4 - t3

    def run(self, requests, idle_sleep: float = 2e-4):
        """Serve requests, each with its arrival time (seconds from start),
        until every one has been delivered. Returns the results."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        self.now()
        while pending or self.waiting or self.active:
            t = self.now()
            while pending and pending[0].arrival <= t:
                self.submit(pending.popleft())
            if not self.waiting and not self.active:
                time.sleep(min(idle_sleep, max(0.0, pending[0].arrival - t)) if pending else 0)
                continue
            self.step()
        return self.results

    def close(self):
        self.pool.close()


def summarize(results, wall_s: float, offspring: int, host_s: dict | None = None) -> dict:
    lat = np.array([r.latency for r in results])
    late = np.array([r.lateness for r in results])
    return {"requests": len(results),
            "p50_time_to_front_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_time_to_front_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "p50_past_deadline_s": float(np.percentile(late, 50)) if len(late) else None,
            "p99_past_deadline_s": float(np.percentile(late, 99)) if len(late) else None,
            "mean_generations": float(np.mean([r.generations for r in results])) if results else 0,
            "offspring_per_s": offspring / wall_s if wall_s > 0 else None,
            "wall_s": wall_s,
            "host_s": dict(host_s) if host_s else None,
            "igd_at_deadline": _stats([r.igd for r in results if r.igd is not None]),
            "hv_at_deadline": _stats([r.hv for r in results if r.hv is not None])}


def _stats(v):
    if not v:
        return None
    a = np.asarray(v, dtype=np.float64)
    return {"count": int(a.size), "median": float(np.median(a)), "mean": float(np.mean(a)),
            "p90": float(np.percentile(a, 90))}
