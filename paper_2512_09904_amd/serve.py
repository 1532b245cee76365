"""Continuous-batching server for parameter-sweep solves (shaft speed, immersion, viscosity).

Requests arrive over time (Poisson arrivals in the sweep workload).  A
request is admitted into a slot of the HIP pool as soon as a slot and enough
of the HBM budget are free; its particle state stays resident on the GPU
until it finishes.  Admitted solves advance together: every pool step is
one batched launch sequence (a captured hipGraph per slot composition) over
the stepped slots, so work of requests that arrived at different times
overlaps on the device.  Which admitted slots are stepped is the policy:
"all" steps every one (processor sharing); "shortest" orders them by
remaining time less a credit for time waited, steps the first one and those
that fit beside it without slowing it beyond a bound, and holds the rest
(see `shortest_first`).
Finished slots are released at once and queued requests take their place.
Each solve's result does not depend on its neighbours in the batch, nor on
when it was held (slot-aligned blocks, deterministic reductions).
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import List, Optional

import numpy as np

from . import cases, sph


@dataclasses.dataclass(eq=False)
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    case: "cases.Case"
    steps: int
    admitted: Optional[float] = None
    finished: Optional[float] = None
    report: Optional[dict] = None
    slot: Optional[int] = None
    remaining: int = 0      # advection steps not yet enqueued
    held: bool = False

    @property
    def latency(self):
        return None if self.finished is None else self.finished - self.arrival


def sweep_requests(n=64, seed=64, steps=500, nf_lo=5e4, nf_hi=2e6, rate=None, scale=1.0):
    """The parameter-sweep workload: U(150, 600) rad/s, immersion U(20, 60) mm,
    nu U(0.5, 3)e-4, fluid count log-uniform in [nf_lo, nf_hi], Poisson arrivals.

    `scale` multiplies the particle counts (small runs for tests).  Without
    `rate` every arrival time is 0 (the caller sets them).
    """
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for k in range(n):
        om = float(rng.uniform(150.0, 600.0))
        imm = float(rng.uniform(0.020, 0.060))
        nu = float(rng.uniform(0.5e-4, 3e-4))
        nf = int(math.exp(rng.uniform(math.log(nf_lo), math.log(nf_hi))) * scale)
        if rate is not None:
            t += float(rng.exponential(1.0 / rate))
        c = cases.serving_tank(max(nf, 2000), om, imm, nu, seed=k)
        reqs.append(Request(rid=k, arrival=t if rate is not None else 0.0, case=c, steps=steps))
    return reqs


# time of one advection step of a slot of n fluid particles stepped alone:
# STEP_COST[0] + STEP_COST[1] * n seconds (serving tank on one MI355X; the
# fixed part is the launch sequence, the rest the sweeps)
STEP_COST = (0.57e-3, 3.3e-9)


def priority(r: Request, now: float, aging: float, cost=STEP_COST) -> float:
    """Scheduling key of the "shortest" policy (smaller first): the request's
    remaining time if it ran alone, less `aging` times the time since it
    arrived, so a long request that has waited gains on newer short ones."""
    return r.remaining * (cost[0] + cost[1] * r.case.nf) - aging * (now - r.arrival)


def shortest_first(active: dict, fill: int, now: float = 0.0, aging: float = 0.0, slowdown: float = 0.0,
                   cost=STEP_COST) -> set:
    """Slots to step under the "shortest" policy.  The admitted requests are
    taken in order of `priority` (ties by arrival, then slot): the first one
    always, each next one only if the batched step stays within the larger
    of (1 + slowdown) times the first one's step alone and the step of
    `fill` particles (small requests share the device freely, a large one
    does not slow a small one down).  A request whose steps are all enqueued
    is neither stepped nor held (it is finishing on the device)."""
    order = sorted(((s, r) for s, r in active.items() if r.remaining > 0),
                   key=lambda kv: (priority(kv[1], now, aging, cost), kv[1].arrival, kv[0]))
    run, acc, limit = set(), 0, 0.0
    for slot, r in order:
        if not run:
            limit = max((1.0 + slowdown) * (cost[0] + cost[1] * r.case.nf), cost[0] + cost[1] * fill)
        elif cost[0] + cost[1] * (acc + r.case.nf) > limit:
            continue
        run.add(slot)
        acc += r.case.nf
    return run


class Server:
    """Admits requests by HBM budget and free slots; steps the admitted slots
    that the policy picks ("all" or "shortest", see the module text)."""

    def __init__(self, hbm_budget: int, max_slots: int = 16, precision: str = "mixed",
                 steps_per_call: int = 10, graph: bool = True, pool=None, policy: str = "all",
                 fill: int = 500_000, slowdown: float = 0.5, aging: float = 4.0, cost=STEP_COST):
        if policy not in ("all", "shortest"):
            raise ValueError(f"unknown policy {policy!r}")
        self.pool = pool if pool is not None else sph.Pool(hbm_budget, max_slots=max_slots,
                                                           precision=precision, graph=graph)
        self.policy = policy
        self.fill = int(fill)
        self.slowdown = float(slowdown)
        self.aging = float(aging)
        self.cost = cost
        self.precision = precision
        self.k = steps_per_call
        self.max_slots = max_slots
        self.budget = hbm_budget
        self.peak_bytes = 0
        self.peak_active = 0

    def run(self, requests: List[Request], clock=time.perf_counter, max_in_flight: int = 2, progress=None):
        """Serve every request; fills admitted/finished/report on each.

        At most `max_in_flight` pool-step calls are queued on the device, so
        admissions and completions are seen within a few calls.
        """
        torch = getattr(self.pool, "torch", None)
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue: collections.deque = collections.deque()
        active = {}
        inflight: collections.deque = collections.deque()
        t0 = clock()
        while pending or queue or active:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            while queue:
                # "all": arrival order; "shortest": priority order
                if self.policy == "all":
                    r = queue[0]
                else:
                    for q in queue:
                        q.remaining = q.steps
                    r = min(queue, key=lambda q: (priority(q, now, self.aging, self.cost), q.arrival))
                if self.pool.bytes_required(r.case, self.precision) > self.budget:
                    raise ValueError(f"request {r.rid} can never fit the HBM budget")
                slot = self.pool.admit(r.case, r.steps)
                if slot is None:
                    break
                queue.remove(r)
                r.slot = slot
                r.admitted = clock() - t0
                r.remaining = r.steps
                r.held = False
                active[slot] = r
            used, nact = self.pool.usage()
            self.peak_bytes = max(self.peak_bytes, used)
            self.peak_active = max(self.peak_active, nact)
            if active:
                if self.policy == "shortest":
                    run = shortest_first(active, self.fill, clock() - t0, self.aging, self.slowdown, self.cost)
                    for slot, r in active.items():
                        want = slot not in run
                        if r.held != want:
                            self.pool.hold(slot, want)
                            r.held = want
                self.pool.step(self.k)
                for r in active.values():
                    if not r.held:
                        r.remaining = max(0, r.remaining - self.k)
                if torch is not None:
                    ev = torch.cuda.Event()
                    ev.record(self.pool.stream)
                    inflight.append(ev)
                    while len(inflight) > max_in_flight:
                        inflight.popleft().synchronize()
                # finished slots (their work has completed on the device)
                for slot in list(active):
                    done, rep = self.pool.poll(slot)
                    if done:
                        r = active.pop(slot)
                        r.finished = clock() - t0
                        r.report = rep
                        r.final = self.pool.get_fluid(slot) if getattr(r, "keep_state", False) else None
                        self.pool.release(slot)
                        if progress is not None:
                            progress(r, len(active), len(queue), len(pending))
            elif pending:
                time.sleep(max(0.0, min(0.01, pending[0].arrival - (clock() - t0))))
        if torch is not None:
            self.pool.stream.synchronize()
        return requests

    def close(self):
        self.pool.close()


def summarize(requests: List[Request], wall: float):
    lat = np.array([r.latency for r in requests])
    pstep = sum(r.case.nf * r.steps for r in requests)
    return dict(n=len(requests), p50_s=float(np.percentile(lat, 50)), p95_s=float(np.percentile(lat, 95)),
                p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()), wall_s=wall,
                particle_steps_per_s=pstep / wall,
                faults=sum(1 for r in requests if r.report and r.report.get("rc", 0) != 0))
