"""Serving scheduler on the CPU, against a stand-in pool with the same interface.

Checks the continuous-batching loop itself: admission only when a slot and
budget are free, FIFO order of queued requests, every request finishes with
its own report, budget never exceeded, a faulted slot is released without
stopping the others.
"""
import numpy as np

from paper_2512_09904_amd import cases, serve


class FakePool:
    """Steps requests by count; 'bytes' per request is its fluid count."""

    def __init__(self, budget, max_slots, fault_rid=None):
        self.budget, self.max_slots = budget, max_slots
        self.slots = {}
        self.used = 0
        self.peak = 0
        self.fault_rid = fault_rid
        self.admit_order = []

    @staticmethod
    def bytes_required(case, precision="mixed"):
        return case.nf

    def admit(self, case, steps):
        need = case.nf
        if len(self.slots) >= self.max_slots or self.used + need > self.budget:
            return None
        s = next(k for k in range(self.max_slots) if k not in self.slots)
        self.slots[s] = dict(case=case, steps=steps, done=0, need=need)
        self.used += need
        self.peak = max(self.peak, self.used)
        self.admit_order.append(case.meta["rid"])
        return s

    def step(self, n):
        for s in self.slots.values():
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
