"""Serving scheduler on the CPU, against a stand-in pool with the same interface.

Checks the continuous-batching loop itself: admission only when a slot and
budget are free, FIFO order of queued requests, every request finishes with
its own report, budget never exceeded, a faulted slot is released without
stopping the others; the "shortest" policy steps the least remaining work
first, up to the fill, and holds the rest.
"""
import numpy as np

from paper_2512_09904_amd import cases, serve


class FakePool:
    """Steps requests by count; 'bytes' per request is its fluid count."""

    def __init__(self, budget, max_slots, fault_rid=None, rate=None):
        self.budget, self.max_slots = budget, max_slots
        self.slots = {}
        self.used = 0
        self.peak = 0
        self.fault_rid = fault_rid
        self.admit_order = []
        self.rate = rate        # particle-steps per unit of virtual time, once the device is full
        self.fill = 0
        self.time = 0.0
        self.stepped = []       # rids stepped by each call

    @staticmethod
    def bytes_required(case, precision="mixed"):
        return case.nf

    def admit(self, case, steps):
        need = case.nf
        if len(self.slots) >= self.max_slots or self.used + need > self.budget:
            return None
        s = next(k for k in range(self.max_slots) if k not in self.slots)
        self.slots[s] = dict(case=case, steps=steps, done=0, need=need, held=False)
        self.used += need
        self.peak = max(self.peak, self.used)
        self.admit_order.append(case.meta["rid"])
        return s

    def hold(self, slot, hold=True):
        self.slots[slot]["held"] = bool(hold)

    def step(self, n):
        run = [s for s in self.slots.values() if not s["held"] and s["done"] < s["steps"]]
        self.stepped.append(sorted(s["case"].meta["rid"] for s in run))
        if self.rate and run:
            # a step takes as long as a full device's step unless more is stepped
            self.time += n * max(self.fill, sum(s["need"] for s in run)) / self.rate
        for s in run:
            s["done"] = min(s["steps"], s["done"] + n)

    def poll(self, slot):
        s = self.slots[slot]
        rc = 6 if s["case"].meta["rid"] == self.fault_rid and s["done"] > 0 else 0
        if s["done"] >= s["steps"] or rc:
            return True, dict(rc=rc, step=s["done"], rid=s["case"].meta["rid"])
        return False, None

    def get_fluid(self, slot):
        return None

    def release(self, slot):
        self.used -= self.slots.pop(slot)["need"]

    def usage(self):
        return self.used, len(self.slots)


def _requests(sizes, steps, arrivals):
    reqs = []
    for k, (n, st, a) in enumerate(zip(sizes, steps, arrivals)):
        c = cases.Case("fake", {}, [], np.zeros((n, 3)), np.zeros((n, 3)), np.zeros(n), np.zeros(n),
                       np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, np.int32), meta=dict(rid=k))
        reqs.append(serve.Request(rid=k, arrival=a, case=c, steps=st))
    return reqs


def test_admission_by_budget_and_fifo():
    pool = FakePool(budget=100, max_slots=3)
    srv = serve.Server(100, max_slots=3, pool=pool, steps_per_call=5)
    reqs = _requests([60, 50, 30, 20, 90], [20, 10, 15, 5, 10], [0, 0, 0, 0, 0])
    srv.run(reqs)
    assert all(r.report is not None and r.report["rid"] == r.rid for r in reqs)
    assert all(r.report["step"] == r.steps for r in reqs)
    assert pool.peak <= 100
    # request 1 (50) waits for request 0 (60) to free budget: FIFO keeps later ones waiting too
    assert pool.admit_order == [0, 1, 2, 3, 4]
    assert reqs[1].admitted >= reqs[0].finished
    assert reqs[2].admitted >= reqs[1].admitted


def test_faulted_request_is_released_and_others_finish():
    pool = FakePool(budget=1000, max_slots=4, fault_rid=1)
    srv = serve.Server(1000, max_slots=4, pool=pool, steps_per_call=2)
    reqs = _requests([10, 10, 10], [8, 8, 8], [0, 0, 0])
    srv.run(reqs)
    assert reqs[1].report["rc"] == 6
    assert reqs[0].report["rc"] == 0 and reqs[2].report["rc"] == 0
    assert pool.used == 0 and not pool.slots


def test_sweep_request_distribution():
    reqs = serve.sweep_requests(n=12, seed=3, steps=5, nf_lo=2000, nf_hi=20000)
    om = [r.case.meta["omega"] for r in reqs]
    imm = [r.case.meta["immersion"] for r in reqs]
    nu = [r.case.meta["nu"] for r in reqs]
    assert all(150 <= w <= 600 for w in om)
    assert all(0.020 <= d <= 0.060 for d in imm)
    assert all(0.5e-4 <= v <= 3e-4 for v in nu)
    assert len({r.case.nf for r in reqs}) > 6


def _active(sizes, remaining):
    reqs = _requests(sizes, remaining, [0.0] * len(sizes))
    for r, left in zip(reqs, remaining):
        r.remaining = left
    return {10 + k: r for k, r in enumerate(reqs)}


def test_shortest_first_takes_least_work_up_to_the_fill():
    # with a cost of one unit per particle-step, work: 4000, 1500, 1000, 6000;
    # order 12 (50 particles), 11 (300), 10 (100), 13 (200)
    act = _active([100, 300, 50, 200], [40, 5, 20, 30])
    pick = lambda a, fill, **kw: serve.shortest_first(a, fill, cost=(0.0, 1.0), **kw)
    assert pick(act, 250) == {12, 10}          # 50, +300 > 250 skipped, +100 = 150, +200 > 250 skipped
    assert pick(act, 50) == {12}
    assert pick(act, 10 ** 9) == set(act)
    # a request joins only if the batched step stays within the larger of
    # (1 + slowdown) x the first one's step alone and the step of `fill`
    act2 = _active([50, 400, 40, 10], [2, 5, 5, 5])    # work 100, 2000, 200, 50: order 13, 10, 12, 11
    assert pick(act2, 0, slowdown=1.0) == {13}          # 10 + 50, 10 + 40, 10 + 400 all > 2 x 10
    assert pick(act2, 0, slowdown=5.0) == {13, 10}      # 60 <= 6 x 10; then 100 > 60
    assert pick(act2, 55) == {13, 12}                   # limit 55: 60 no, 50 yes, 450 no
    assert pick(act2, 55, slowdown=1e9) == set(act2)
    # a request with no steps left is finishing: neither stepped nor counted
    act[12].remaining = 0
    assert pick(act, 250) == {11}
    # equal work: the earlier arrival first
    act = _active([100, 100], [10, 10])
    act[10].arrival, act[11].arrival = 2.0, 1.0
    assert pick(act, 100) == {11}
    assert pick({}, 100) == set()
    # aging: a long request that has waited overtakes a newer short one
    act = _active([1, 1], [100, 50])
    act[10].arrival, act[11].arrival = 0.0, 10.0
    assert pick(act, 0, now=10.0) == {11}
    assert pick(act, 0, now=10.0, aging=10.0) == {10}
    assert serve.priority(act[10], 10.0, 10.0, cost=(0.0, 1.0)) == 0.0
    assert serve.priority(act[11], 10.0, 10.0, cost=(2.0, 1.0)) == 150.0


def test_shortest_policy_finishes_small_requests_first():
    """Two large (500) and two small (100) requests of ten steps arrive
    together on a device that is full at 100 particles (1000 particle-steps
    per time unit).  Stepping everything together (processor sharing)
    finishes all four at 10 x 1200 / 1000 = 12; the shortest policy steps one
    request at a time, each filling the device, smallest first: they finish
    at 1, 2, 7 and 12, the same total time, every request complete."""
    def run(policy):
        pool = FakePool(budget=10 ** 9, max_slots=8, rate=1000.0)
        pool.fill = 100
        srv = serve.Server(10 ** 9, max_slots=8, pool=pool, steps_per_call=10, policy=policy, fill=100,
                           slowdown=0.0, aging=0.0)
        reqs = _requests([500, 500, 100, 100], [10, 10, 10, 10], [0.0] * 4)
        srv.run(reqs, clock=lambda: pool.time)
        assert all(r.report["step"] == 10 for r in reqs)
        return reqs, pool

    reqs, pool = run("all")
    assert [r.finished for r in reqs] == [12.0] * 4
    assert pool.stepped[0] == [0, 1, 2, 3]
    reqs, pool = run("shortest")
    assert [r.finished for r in reqs] == [7.0, 12.0, 1.0, 2.0]
    assert pool.stepped == [[2], [3], [0], [1]]
    assert pool.time == 12.0


def test_shortest_policy_admits_the_smallest_queued_request():
    pool = FakePool(budget=100, max_slots=1)
    srv = serve.Server(100, max_slots=1, pool=pool, steps_per_call=5, policy="shortest", fill=10, aging=0.0)
    reqs = _requests([60, 50, 30, 20], [10, 10, 10, 10], [0, 0, 0, 0])
    srv.run(reqs)
    assert pool.admit_order == [3, 2, 1, 0]
    assert all(r.report["step"] == 10 for r in reqs)


def test_unknown_policy_is_refused():
    import pytest
    with pytest.raises(ValueError):
        serve.Server(100, pool=FakePool(100, 1), policy="lifo")
