"""Serving pool on the GPU: batched solves equal solo solves, admission by budget.

Each request's result must be identical (bitwise) whether it runs alone or
batched with others admitted at different times, since slots own whole
blocks and every reduction has a fixed order.
"""
import ctypes
import sys
import time

import numpy as np
import pytest

from paper_2512_09904_amd import cases

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sph():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_09904_amd import sph as S
    S.lib()
    return S


def _wait(pool, slot, tries=500):
    for _ in range(tries):
        done, rep = pool.poll(slot)
        if done:
            return rep
        time.sleep(0.005)
    raise AssertionError(f"slot {slot} did not finish")


def _requests():
    return [cases.serving_tank(6000, 300.0, 0.03, 1e-4, seed=1),
            cases.serving_tank(9000, 450.0, 0.045, 2e-4, seed=2),
            cases.serving_tank(4000, 200.0, 0.025, 0.7e-4, seed=3)]


def _run_pool(sph, reqs, steps, stagger, max_slots=4, precision="mixed"):
    pool = sph.Pool(1 << 40, max_slots=max_slots, precision=precision)
    out = {}
    slots = {}
    pending = list(range(len(reqs)))
    k = 0
    while pending or slots:
        # admit request q once `stagger[q]` pool steps have been taken
        for q in list(pending):
            if stagger[q] <= k:
                s = pool.admit(reqs[q], steps[q])
                if s is not None:
                    slots[s] = q
                    pending.remove(q)
        pool.step(1)
        k += 1
        for s in list(slots):
            done, rep = pool.poll(s)
            if done:
                q = slots.pop(s)
                out[q] = (pool.get_fluid(s), rep)
                pool.release(s)
        if k > 1000:
            raise RuntimeError("pool did not drain")
    pool.close()
    return out


def test_alone_equals_in_mix(sph):
    reqs = _requests()
    steps = [7, 5, 9]
    say("serving: alone vs mix")
    alone = {q: _run_pool(sph, [reqs[q]], [steps[q]], [0])[0] for q in range(3)}
    mix = _run_pool(sph, reqs, steps, [0, 2, 3])
    for q in range(3):
        ga, ra = alone[q]
        gm, rm = mix[q]
        assert ra["rc"] == 0 and rm["rc"] == 0
        assert ra["step"] == steps[q] == rm["step"]
        for key in ("x", "v", "rho", "T"):
            assert np.array_equal(ga[key], gm[key]), (q, key)
        assert ra["bodies"][1]["torque_axis"] == rm["bodies"][1]["torque_axis"]
        assert ra["heat_total"] == rm["heat_total"]



def test_held_slot_is_unchanged_and_resumes_to_its_solo_result(sph):
    """A held slot is left out of pool steps: its state and report do not
    move while the others step, it does not finish, and once resumed it ends
    bitwise where its solo run ends; the slots stepped meanwhile are not
    disturbed either."""
    reqs = _requests()
    steps = [6, 8, 5]
    say("serving: hold and resume")
    alone = {q: _run_pool(sph, [reqs[q]], [steps[q]], [0])[0] for q in range(3)}
    pool = sph.Pool(1 << 40, max_slots=4)
    slots = [pool.admit(reqs[q], steps[q]) for q in range(3)]
    pool.step(2)
    pool.hold(slots[0])
    pool.hold(slots[2])
    before = [pool.get_fluid(slots[q]) for q in (0, 2)]
    pool.step(3)                      # only request 1 steps
    after = [pool.get_fluid(slots[q]) for q in (0, 2)]
    for b, a in zip(before, after):
        for key in ("x", "v", "rho", "T"):
            assert np.array_equal(a[key], b[key]), key
    assert not pool.poll(slots[0])[0] and not pool.poll(slots[2])[0]
    pool.hold(slots[1])               # every slot held: a step does nothing
    mid = pool.get_fluid(slots[1])
    pool.step(2)
    assert all(np.array_equal(pool.get_fluid(slots[1])[k], mid[k]) for k in ("x", "v", "rho", "T"))
    pool.hold(slots[0], False)
    pool.hold(slots[0], False)        # resuming twice is harmless
    pool.hold(slots[1], False)
    pool.hold(slots[2], False)
    pool.step(max(steps))             # more than any slot has left: finished slots drop out
    out = {}
    for q in range(3):
        rep = _wait(pool, slots[q])
        out[q] = (pool.get_fluid(slots[q]), rep)
    for q in range(3):
        ga, ra = alone[q]
        gm, rm = out[q]
        assert rm["rc"] == 0 and rm["step"] == steps[q] == ra["step"]
        for key in ("x", "v", "rho", "T"):
            assert np.array_equal(ga[key], gm[key]), (q, key)
        assert ra["bodies"][1]["torque_axis"] == rm["bodies"][1]["torque_axis"]
        assert ra["heat_total"] == rm["heat_total"] and ra["t"] == rm["t"]
    # a slot that is not in use, and a flag other than 0 or 1, are refused
    pool.release(slots[1])
    with pytest.raises(sph.SphError) as e:
        pool.hold(slots[1])
    assert e.value.code == sph.SPH_ERR_ARG
    rc = sph.lib().sph_pool_hold(pool.h, ctypes.c_int32(slots[0]), ctypes.c_int32(2))
    assert rc == sph.SPH_ERR_ARG
    pool.close()


def test_alone_equals_in_mix_with_viscous_heating(sph):
    """The middle request has viscous dissipation heating (eq. 23) on, so the
    batched viscous launch takes its dissipation variant for every slot; each
    request still matches its solo run bitwise, and only the heated one
    reports dissipated heat."""
    reqs = _requests()
    reqs[1].params = dict(reqs[1].params, viscous_heating=1)
    steps = [6, 5, 4]
    say("serving: alone vs mix, one slot with viscous heating")
    alone = {q: _run_pool(sph, [reqs[q]], [steps[q]], [0])[0] for q in range(3)}
    mix = _run_pool(sph, reqs, steps, [0, 1, 1])
    for q in range(3):
        ga, ra = alone[q]
        gm, rm = mix[q]
        assert ra["rc"] == 0 and rm["rc"] == 0
        for key in ("x", "v", "rho", "T"):
            assert np.array_equal(ga[key], gm[key]), (q, key)
        assert ra["diss_total"] == rm["diss_total"]
        assert (rm["diss_total"] > 0.0) == (q == 1)


def test_alone_equals_in_mix_with_materials(sph):
    """The middle request carries two fluid materials, so the batched viscous
    launch takes its material variant for every slot; each request still
    matches its solo run bitwise."""
    reqs = _requests()
    r = reqs[1]
    r.params = dict(r.params, materials=[(0.13, 2000.0), (0.4, 1500.0)])
    r.material = (r.xf[:, 0] > r.xf[:, 0].mean()).astype(np.int32)
    steps = [5, 4, 6]
    say("serving: alone vs mix, one slot with two materials")
    alone = {q: _run_pool(sph, [reqs[q]], [steps[q]], [0])[0] for q in range(3)}
    mix = _run_pool(sph, reqs, steps, [0, 1, 2])
    for q in range(3):
        ga, ra = alone[q]
        gm, rm = mix[q]
        assert ra["rc"] == 0 and rm["rc"] == 0
        for key in ("x", "v", "rho", "T"):
            assert np.array_equal(ga[key], gm[key]), (q, key)
        assert ra["thermal"] == rm["thermal"]

def test_solver_equals_pool_slot(sph):
    c = _requests()[0]
    say("serving: solver vs pool")
    s = sph.Solver(c)
    s.step(5)
    r = s.reduce()
    g = s.get_fluid()
    s.close()
    gp, rp = _run_pool(sph, [c], [5], [0])[0]
    for key in ("x", "v", "rho", "T"):
        assert np.array_equal(g[key], gp[key]), key
    assert r["bodies"][1]["torque_axis"] == rp["bodies"][1]["torque_axis"]


def test_fp64_pool_mix_equals_fp64_solver(sph):
    """In FP64 mode too, a request batched with others gives the solver's
    own result bit for bit."""
    reqs = _requests()
    say("serving: fp64 pool mix vs fp64 solver")
    s = sph.Solver(reqs[2], precision="fp64")
    s.step(4)
    r = s.reduce()
    g = s.get_fluid()
    s.close()
    mix = _run_pool(sph, reqs, [3, 5, 4], [0, 1, 1], precision="fp64")
    gm, rm = mix[2]
    assert rm["rc"] == 0 and rm["step"] == 4
    for key in ("x", "v", "rho", "T"):
        assert np.array_equal(g[key], gm[key]), key
    assert r["thermal"] == rm["thermal"] and r["heat_total"] == rm["heat_total"]


@pytest.mark.parametrize("policy", ["all", "shortest"])
def test_server_results_equal_solo_runs(sph, policy):
    """The continuous-batching server with each policy over six requests of
    different sizes and step counts, at most three slots: every request's
    final state and report equal its solo run bit for bit, whatever it was
    batched with and however often the "shortest" policy held it (its fill
    of 8,000 particles holds the larger requests behind the smaller ones)."""
    from paper_2512_09904_amd import serve
    cs = [cases.serving_tank(n, om, imm, nu, seed=k) for k, (n, om, imm, nu) in
          enumerate([(9000, 300.0, 0.04, 1e-4), (3000, 450.0, 0.03, 2e-4), (6000, 200.0, 0.05, 1.5e-4),
                     (2500, 350.0, 0.035, 1e-4), (7000, 500.0, 0.045, 2.5e-4), (4000, 250.0, 0.025, 0.8e-4)])]
    steps = [12, 6, 9, 5, 8, 7]
    say("serving: server", policy)
    alone = [_run_pool(sph, [c], [n], [0])[0] for c, n in zip(cs, steps)]
    reqs = [serve.Request(rid=k, arrival=0.0, case=c, steps=n) for k, (c, n) in enumerate(zip(cs, steps))]
    for r in reqs:
        r.keep_state = True
    srv = serve.Server(1 << 40, max_slots=3, steps_per_call=2, policy=policy, fill=8000)
    srv.run(reqs)
    srv.close()
    for r, (ga, ra) in zip(reqs, alone):
        assert r.report["rc"] == 0 and r.report["step"] == r.steps == ra["step"]
        for key in ("x", "v", "rho", "T"):
            assert np.array_equal(r.final[key], ga[key]), (r.rid, key)
        assert r.report["bodies"][1]["torque_axis_int"] == ra["bodies"][1]["torque_axis_int"]
        assert r.report["heat_total"] == ra["heat_total"] and r.report["t"] == ra["t"]
    assert srv.peak_active <= 3


def test_admission_respects_budget(sph):
    reqs = _requests()
    need = [sph.Pool.bytes_required(c) for c in reqs]
    budget = need[0] + need[2] + 1
    say("serving: budget", need, budget)
    pool = sph.Pool(budget, max_slots=8)
    s0 = pool.admit(reqs[0], 3)
    assert s0 is not None
    assert pool.admit(reqs[1], 3) is None          # does not fit next to request 0
    s2 = pool.admit(reqs[2], 3)
    assert s2 is not None
    used, active = pool.usage()
    assert used <= budget and active == 2
    pool.step(3)
    for s in (s0, s2):
        rep = _wait(pool, s)
        assert rep["rc"] == 0 and rep["step"] == 3
        pool.release(s)
    assert pool.admit(reqs[1], 3) is not None       # admitted once budget is free
    pool.close()


def test_faulted_slot_does_not_disturb_others(sph):
    reqs = _requests()
    bad = reqs[1].copy()
    bad.xf[10] = [1.0, 1.0, 1.0]   # outside the grid: this solve faults at its first step
    say("serving: fault isolation")
    ref = _run_pool(sph, [reqs[0]], [4], [0])[0]
    pool = sph.Pool(1 << 40, max_slots=4)
    a = pool.admit(reqs[0], 4)
    b = pool.admit(bad, 4)
    pool.step(4)
    rep_b = _wait(pool, b)
    assert rep_b["rc"] == sph.SPH_ERR_DOMAIN
    rep_a = _wait(pool, a)
    assert rep_a["rc"] == 0 and rep_a["step"] == 4
    g = pool.get_fluid(a)
    for key in ("x", "v", "rho", "T"):
        assert np.array_equal(g[key], ref[0][key])
    pool.close()


def test_poll_right_after_admit_sees_a_clean_slot(sph):
    """A poll issued before the admitted slot's upload has run on the pool's
    stream must wait for it, not read what the reused memory held before
    (here a freed block of -1 words under a busy stream)."""
    import torch
    pool = sph.Pool(1 << 40, max_slots=2)
    with torch.cuda.stream(pool.stream):
        junk = torch.full((64 << 20,), -1, dtype=torch.int32, device="cuda")
        del junk
        torch.cuda._sleep(20_000_000)               # keep the pool's stream busy for a while
    c = cases.serving_tank(4000, 200.0, 0.025, 0.7e-4, seed=3)
    s = pool.admit(c, 2)
    done, rep = pool.poll(s)
    assert not done, rep
    pool.step(2)
    rep = _wait(pool, s)
    assert rep["rc"] == 0 and rep["step"] == 2
    pool.close()
