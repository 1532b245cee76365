"""Benchmark of the WCSPH gearbox hot path on one MI355X.

Workload: the 1.5 mm gearbox proxy (two meshing toothed disks, 20/40 teeth,
module 4 mm, 300 rad/s, 30 mm immersion, nu = 1e-4; about 0.89 M fluid and
0.48 M solid particles), synthetic seeded input, mixed FP32/FP64 arithmetic.

A step is one advection step of the whole hot path: body pose, cell sort,
neighbour rows, density re-initialisation, time step, viscous + heat sweep,
n_ac acoustic sub-steps (momentum and continuity sweeps) and the reductions.

Printed: one JSON line with particle-interactions/s (ordered pairs within 2h
times pair sweeps per step), steps/s, per-sweep latency percentiles, the
roofline of the dominant kernel and the FP64 oracle's rate on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# the solver kernels' sources: the HBM-traffic record is valid only for these exact texts
KERNEL_SRC = [os.path.join(ROOT, "paper_2512_09904_amd", "csrc", f)
              for f in ("sph_kernels.hip", "sph_device.h", "sph_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_gearbox_c2.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pair_counts(s, nf):
    cnt = s.dump("nbr_count").reshape(2, nf).astype(np.int64)
    return int(cnt[0].sum()), int(cnt[1].sum())


def sweep_bytes(kernel, nf, nsr, pf, ps, prec="mixed"):
    """Algorithmic HBM bytes of one launch: each array touched once, rows streamed.

    `nsr` is the number of distinct solid particles that appear in some
    fluid particle's row (the wall arrays read).  A row entry is the
    neighbour's 4-byte index; the pair vector comes from the cell-relative
    positions (one 4-wide record per particle).  The neighbour-state gathers
    re-read arrays already counted once.
    """
    rb = 8 if prec == "fp64" else 4          # Real
    pb = 4 if prec == "fp32" else 8          # Pos, Temp
    v4 = 4 * rb
    rows = (pf + ps) * 4
    cnt = 8                                  # fluid and solid row lengths
    if kernel == "momentum":
        # vr, offsets, ah, counts read; vrn written; drift read and written; wall offsets, lever arms
        return nf * (v4 + v4 + v4 + cnt + v4 + 2 * v4) + rows + nsr * 2 * v4
    if kernel == "continuity":
        # vrn, offsets, counts read; drho and vr written; wall offsets, normals, velocities
        return nf * (v4 + v4 + cnt + rb + v4) + rows + nsr * 3 * v4
    if kernel == "visc_heat":
        # with the first sub-step's momentum: vr, offsets, T, Drho, the 16-byte (T, Drho) records
        # of the neighbour gathers, counts read; ah and vrn written; drift read and written; wall
        # offsets, dummy velocities, lever arms
        return nf * (v4 + v4 + pb + rb + 16 + cnt + v4 + v4 + 2 * v4) + rows + nsr * 3 * v4
    if kernel == "build":
        # anchors read; offsets and counts written; rows written (the particle-major staging is
        # read back from cache); wall positions
        return nf * (4 * pb + v4 + cnt) + rows + nsr * 4 * pb
    if kernel == "sumw":
        # anchors, counts read; sum W written; vr read and written; rows read; wall positions
        return nf * (4 * pb + cnt + 8 + 2 * v4) + rows + nsr * 4 * pb
    raise KeyError(kernel)


MODEL_TEXT = {"build": "20 B x {p:.2f} + 40 B",
              "visc_heat": "8 B x {p:.2f} + 50 B, plus 20 B x {p:.2f} + 60 B for the first sub-step's momentum",
              "momentum": "20 B x {p:.2f} + 60 B", "continuity": "20 B x {p:.2f} + 60 B"}


def model_bytes(kernel, nf, pbar):
    """Algorithmic bytes of one launch in the hot-path byte model: per fluid
    particle, 20 B per ordered pair (a frozen pair record: neighbour index,
    pair vector, kernel gradient) plus the particle's own state.  pbar is the
    measured mean of ordered pairs (fluid and solid neighbours) per fluid
    particle.  The kernel sum is fused into the build in that model, so it
    has no entry of its own.  The viscous/heat sweep also runs the first
    acoustic sub-step's momentum, so it is charged both sweeps' bytes."""
    per = {"build": 20.0 * pbar + 40.0, "visc_heat": (8.0 * pbar + 50.0) + (20.0 * pbar + 60.0),
           "momentum": 20.0 * pbar + 60.0, "continuity": 20.0 * pbar + 60.0}.get(kernel)
    return None if per is None else nf * per


def build_candidates(s, case):
    """Candidate pairs of a 27-cell stencil search: for every fluid particle,
    the fluid and solid particles in its own and the 26 adjacent cells of
    edge 2h (the minimum the cell-list method tests, whatever the kernel's
    traversal).  Cells from the current FP64 positions."""
    p = case.params
    cs = 2.0 * p["h_over_dp"] * p["dp"]
    lo = np.asarray(p["grid_lo"], dtype=np.float64)
    hi = np.asarray(p["grid_hi"], dtype=np.float64)
    dims = np.floor((hi - lo) / cs).astype(np.int64) + 1
    xf = s.get_fluid()["x"]
    xs = s.dump("solid_state").reshape(case.ns, 13)[:, 0:3]

    def occupancy(x):
        c = np.clip(np.floor((x - lo) / cs).astype(np.int64), 0, dims - 1)
        g = np.zeros(tuple(dims[::-1]), dtype=np.int64)
        np.add.at(g, (c[:, 2], c[:, 1], c[:, 0]), 1)
        return g, c

    gf, cf = occupancy(xf)
    gs, _ = occupancy(xs)
    tot = gf + gs
    pad = np.pad(tot, 1)
    nb = sum(pad[1 + dz:1 + dz + tot.shape[0], 1 + dy:1 + dy + tot.shape[1], 1 + dx:1 + dx + tot.shape[2]]
             for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1))
    return int(nb[cf[:, 2], cf[:, 1], cf[:, 0]].sum())


def distinct_wall_particles(s, nf):
    """Solid particles referenced by at least one fluid particle's row."""
    cnt = s.dump("nbr_count").reshape(2, nf)[1].astype(np.int64)
    ks = len(s.dump("nbr_solid")) // nf
    rows = s.dump("nbr_solid").reshape(nf, ks)
    mask = np.arange(ks)[None, :] < cnt[:, None]
    return int(np.unique(rows[mask]).size)


def pct(a, q):
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def cpu_baseline(case, steps=6, threads=None):
    """The FP64 oracle on the host cores (or `threads` of them), on a bounded
    sample of the same workload."""
    from oracle import oracle as O
    O.build(force=False)
    prev = O.set_threads(threads) if threads else None
    mats = case.params.get("materials")
    if mats and case.material is not None:
        m = np.asarray(mats, dtype=np.float64)[case.material]
        o = O.State(case, k=m[:, 0], cp=m[:, 1])
    else:
        o = O.State(case)
    nb = O.Nbr(case.params, case.xf, O.body_pose(case.bodies, case.xs0, case.ns0, case.body, 0.0)[0])
    pf = int(nb.csr(0)[0][-1])
    ps = int(nb.csr(1)[0][-1])
    del nb
    t0 = time.perf_counter()
    nac = []
    for _ in range(steps):
        r = o.step()
        nac.append(r["n_ac"])
    dt = time.perf_counter() - t0
    sweeps = sum(2 + 2 * n for n in nac)
    cores = threads or int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    if prev:
        O.set_threads(prev)
    return {"value": (pf + ps) * sweeps / dt, "unit": "particle-interactions/s", "cores": cores,
            "kind": "oracle", "steps_per_s": steps / dt,
            "sample": f"{steps} advection steps of the full gearbox proxy (dp 1.5 mm, {case.nf} fluid + {case.ns} "
                      f"solid particles) from the initial state, FP64 C/OpenMP oracle, {dt:.1f} s"}


def run_serving(n, steps, scale, budget_gb, slots, seeds, precision="mixed", policies=("all", "shortest")):
    """Parameter-sweep serving: continuous batching vs one solve at a time.

    Requests: shaft speed U(150, 600) rad/s, immersion U(20, 60) mm, nu
    U(0.5, 3)e-4, fluid count log-uniform 50k-2M times `scale`, `steps`
    advection steps each.  Each request's service time alone is measured
    first (one slot); arrivals are Poisson with rate 0.85 / mean service
    time; the one-at-a-time server's latencies follow exactly from the
    measured service times (FIFO); the batched server is run live on the
    same requests and arrival times, once per scheduling policy ("all":
    every admitted solve stepped together; "shortest": shortest remaining
    time first with aging, batched up to the device's fill).
    """
    import torch
    from paper_2512_09904_amd import serve, sph
    budget = int(budget_gb * (1 << 30))
    t0 = time.perf_counter()
    reqs = serve.sweep_requests(n=n, seed=64, steps=steps, scale=scale)
    log(f"generated {len(reqs)} requests in {time.perf_counter() - t0:.1f} s; "
        f"fluid {sum(r.case.nf for r in reqs)} total")
    # service time of each request alone
    svc = []
    for r in reqs:
        pool = sph.Pool(budget, max_slots=1, precision=precision)
        torch.cuda.synchronize()
        a = time.perf_counter()
        slot = pool.admit(r.case, r.steps)
        pool.step(r.steps)
        while True:
            done, rep = pool.poll(slot)
            if done:
                break
            time.sleep(0.0005)
        svc.append(time.perf_counter() - a)
        r.alone = rep
        if len(svc) % 8 == 0:
            log(f"alone: {len(svc)}/{len(reqs)} requests, last {svc[-1]:.3f} s (nf {r.case.nf})")
        pool.release(slot)
        pool.close()
    svc = np.array(svc)
    sbar = float(svc.mean())
    log(f"alone: mean service {sbar:.3f} s, total {svc.sum():.1f} s")
    results = []
    for seed in range(64, 64 + seeds):
        rng = np.random.default_rng(seed)
        rate = 0.85 / sbar
        arr = np.cumsum(rng.exponential(1.0 / rate, len(reqs)))
        arr -= arr[0]
        # one-at-a-time FIFO server on the same GPU: latencies from the service times
        fin = np.zeros(len(reqs))
        free = 0.0
        for k in np.argsort(arr, kind="stable"):
            start = max(arr[k], free)
            fin[k] = start + svc[k]
            free = fin[k]
        lat1 = fin - arr
        entry = dict(seed=seed, rate_per_s=rate,
                     one_at_a_time=dict(p50_s=float(np.percentile(lat1, 50)),
                                        p95_s=float(np.percentile(lat1, 95)),
                                        p99_s=float(np.percentile(lat1, 99)),
                                        wall_s=float(fin.max()),
                                        particle_steps_per_s=float(sum(r.case.nf * r.steps for r in reqs) / fin.max())),
                     batched={}, peak_slots={}, peak_gb={}, results_equal_alone=True)
        for policy in policies:
            for r, a in zip(reqs, arr):
                r.arrival = float(a)
                r.admitted = r.finished = r.report = None
            srv = serve.Server(budget, max_slots=slots, precision=precision, policy=policy)
            a = time.perf_counter()
            ndone = [0]

            def progress(r, nact, nq, npend):
                ndone[0] += 1
                if ndone[0] % 8 == 0:
                    log(f"batched ({policy}): {ndone[0]} done, {nact} active, {nq} queued, {npend} not arrived")

            srv.run(reqs, progress=progress)
            wall = time.perf_counter() - a
            same = all(np.array_equal(r.report["bodies"][1]["torque_axis"], r.alone["bodies"][1]["torque_axis"]) and
                       r.report["heat_total"] == r.alone["heat_total"] for r in reqs)
            entry["batched"][policy] = serve.summarize(reqs, wall)
            entry["peak_slots"][policy] = srv.peak_active
            entry["peak_gb"][policy] = srv.peak_bytes / (1 << 30)
            entry["results_equal_alone"] = entry["results_equal_alone"] and bool(same)
            srv.close()
        results.append(entry)
        log(json.dumps(results[-1]))
    workload = (f"{len(reqs)} serving-tank requests (fluid {sum(r.case.nf for r in reqs)} in total), {steps} steps "
                f"each, Poisson arrivals at 0.85/mean service, budget {budget_gb} GB, {slots} slots, particle "
                f"scale {scale}")
    return dict(workload=workload, mean_service_alone_s=sbar, seeds=results)


def serve_bench(args):
    """The full serving sweep as its own JSON line."""
    res = run_serving(args.serve_n, args.serve_steps, args.serve_scale, args.serve_budget_gb, args.serve_slots,
                      args.serve_seeds)
    b = res["seeds"][0]["batched"]["shortest" if "shortest" in res["seeds"][0]["batched"] else "all"]
    out = {"metric": "serving sweep: p50/p99 time-to-result and throughput, batched vs one at a time",
           "value": b["particle_steps_per_s"], "unit": "fluid particle-steps/s", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic", "dtype": "f32+f64",
           "config": {"workload": res["workload"]},
           "mean_service_alone_s": res["mean_service_alone_s"], "seeds": res["seeds"]}
    print(json.dumps(out), flush=True)


def serve_quick(args):
    """A reduced serving sweep carried in the default line: fewer, smaller
    requests than the full sweep, each arrival seed compared with one at a
    time on the same requests."""
    res = run_serving(args.quick_serve_n, args.quick_serve_steps, args.quick_serve_scale, args.serve_budget_gb,
                      args.serve_slots, args.quick_serve_seeds)
    rows = []
    for e in res["seeds"]:
        o = e["one_at_a_time"]
        keys = ("p50_s", "p95_s", "p99_s", "particle_steps_per_s")
        rows.append({"seed": e["seed"],
                     "batched": {pol: {k: b[k] for k in keys} for pol, b in e["batched"].items()},
                     "one_at_a_time": {k: o[k] for k in keys},
                     "peak_slots": e["peak_slots"], "results_equal_alone": e["results_equal_alone"]})
    return {"workload": res["workload"], "unit": "s (time to result), fluid particle-steps/s",
            "mean_service_alone_s": res["mean_service_alone_s"], "seeds": rows}


def relax_bench(args):
    """Physics-driven particle relaxation (Section 2.2) of the 40-tooth gear
    body of the gearbox proxy: lattice sites inside the level set, jittered by
    +-0.25 dp, relaxed for `relax_iters` iterations after 2 untimed ones."""
    import torch
    from paper_2512_09904_amd import cases, sph
    dp = args.dp
    shape = dict(kind="gear", center=(0.190, 0.075, 0.100), size=(0.084, 0.075, 0.015), teeth=40, phase=0.5)
    c = cases.relax_case(shape, dp, 0.090, jitter_amp=0.25, seed=0)
    log(f"relax case: {c.nf} particles in the 40-tooth gear at dp={dp * 1e3:.2f} mm")
    s = sph.Solver(c, precision=args.precision)
    first = s.relax(shape, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = s.relax(shape, args.relax_iters)
    wall = time.perf_counter() - t0
    s.set_timing(True)
    s.relax(shape, 3)
    kt = {k: float(np.mean(s.timing(k))) for k in ("relax_force", "relax_max", "relax_move", "build", "sumw")
          if len(s.timing(k))}
    s.set_timing(False)
    g = s.get_fluid()
    s.close()
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        O.build(force=False)
        t1 = time.perf_counter()
        x = c.xf
        for _ in range(2):
            x, _, _ = O.relax_step(c.params, shape, x)
        tc = time.perf_counter() - t1
        cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
        cpu = {"value": 2.0 / tc, "unit": "iterations/s", "cores": cores, "kind": "oracle",
               "sample": f"two relaxation iterations of the same {c.nf} particles from the jittered start, "
                         f"FP64 C/OpenMP oracle, {tc:.1f} s"}
    ms = 1e3 * wall / args.relax_iters
    print(json.dumps({"metric": "particle relaxation iterations/s (Section 2.2)", "value": 1e3 / ms,
                      "unit": "iterations/s", "ms_per_iteration": ms, "iterations": args.relax_iters,
                      "particle_iterations_per_s": c.nf * 1e3 / ms, "precision": args.precision,
                      "config": {"workload": f"40-tooth gear body (r_tip 84 mm, r_root 75 mm, face 30 mm) "
                                             f"at dp={dp * 1e3:.2f} mm, jittered lattice start",
                                 "n_particles": c.nf},
                      "kernel_ms": kt, "amax_start": first["amax_first"], "amax_end": rep["amax_last"],
                      "bounded_last": rep["bounded_last"], "cpu_baseline": cpu}), flush=True)


def contact_bench(args):
    """Contact factor (eq. 24) of every solid particle of the gearbox proxy after
    10 steps: the call (cell sort, neighbour build and the solid-centric
    k_contact sweep) timed over `contact_calls` calls."""
    import torch
    from paper_2512_09904_amd import cases, sph
    case = cases.gearbox(seed=0, dp=args.dp, omega_big=300.0, immersion=0.030, nu=1e-4)
    log(f"contact case: nf={case.nf} ns={case.ns}")
    s = sph.Solver(case, precision=args.precision)
    s.step(10)
    s.reduce()
    s.contact_factor()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.contact_calls):
        z, means = s.contact_factor()
    wall = time.perf_counter() - t0
    s.set_timing(True)
    s.contact_factor()
    kt = {k: float(np.mean(s.timing(k))) for k in ("contact", "build", "sumw", "cellsort") if len(s.timing(k))}
    s.set_timing(False)
    t = s.reduce()["t"]
    g = s.get_fluid()
    s.close()
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        O.build(force=False)
        xs, _, _ = O.body_pose(case.bodies, case.xs0, case.ns0, case.body, t)
        t1 = time.perf_counter()
        zo = O.contact_factor(case.params, g["x"], g["rho"], xs)
        tc = time.perf_counter() - t1
        cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
        cpu = {"value": case.ns / tc, "unit": "solid particles/s", "cores": cores, "kind": "oracle",
               "sample": f"one contact-factor evaluation of the same {case.ns} solid particles, FP64 C oracle, "
                         f"{tc:.2f} s", "max_abs_diff_vs_gpu": float(np.max(np.abs(zo - z)))}
    ms = 1e3 * wall / args.contact_calls
    print(json.dumps({"metric": "contact factor evaluations/s (eq. 24)", "value": 1e3 / ms, "unit": "calls/s",
                      "ms_per_call": ms, "solid_particles_per_s": case.ns * 1e3 / ms, "precision": args.precision,
                      "config": {"workload": f"gearbox proxy dp={args.dp * 1e3:.2f} mm after 10 steps",
                                 "n_fluid": case.nf, "n_solid": case.ns},
                      "kernel_ms": kt, "body_means": [float(m) for m in means], "cpu_baseline": cpu}), flush=True)


def precision_study(args):
    """All-FP32 vs mixed FP32/FP64 vs FP64 on the churning tank (C1 geometry).

    Each mode runs the same advection steps (its own adaptive time steps)
    from the same state; the FP64 GPU run is the reference.  At checkpoints
    every `ps_ckpt` steps each mode reports: simulated time, drift of the
    mass proxy sum(rho dp^3) against the exact mass, the heat-balance
    residual (thermal energy change minus the integrated heat inflow, over
    the inflow), the mean oil temperature rise and the time-mean disk torque;
    the comparison with FP64 is made at equal step counts.  A mode that
    faults (a particle leaving the grid, a non-finite value) stops there.
    """
    from paper_2512_09904_amd import cases, sph
    c = cases.tank_c1(dp=args.ps_dp, omega=450.0)
    log(f"precision study: nf={c.nf} ns={c.ns} steps={args.ps_steps}")
    m = c.params["rho0"] * c.params["dp"] ** 3
    cp = c.params["cp_f"]
    E0 = math.fsum(m * cp * c.Tf)
    out = {}
    final = {}
    for mode in ("fp64", "mixed", "fp32"):
        s = sph.Solver(c, precision=mode)
        t0 = time.perf_counter()
        done = 0
        series = []
        fault = None
        while done < args.ps_steps:
            n = min(args.ps_ckpt, args.ps_steps - done)
            s.step(n)
            r = s.reduce(raise_on_fault=False)
            if r["rc"]:
                fault = {"rc": r["rc"], "step": int(r["step"])}
                log(f"{mode}: fault {r['rc']} at step {r['step']}")
                break
            done += n
            dE = r["thermal"] - E0
            series.append({"step": done, "t": r["t"], "mass_proxy_drift": r["mass_proxy"] / r["mass"] - 1.0,
                           "heat_balance_residual": (dE - r["heat_total"]) / abs(r["heat_total"]),
                           "mean_T_rise_K": dE / (m * cp * c.nf),
                           "disk_torque_mean_Nm": r["bodies"][1]["torque_axis_int"] / r["t"]})
            log(f"{mode}: {done} steps, t={r['t']:.4f} s, vmax={r['vmax']:.2f}, "
                f"heat residual {series[-1]['heat_balance_residual']:.2e}")
        wall = time.perf_counter() - t0
        g = s.get_fluid() if fault is None else None
        s.close()
        out[mode] = {"steps_done": done, "wall_s": wall, "fault": fault, "series": series}
        final[mode] = g
        if series:
            log(f"{mode}: {json.dumps(series[-1])}")
    ref = {e["step"]: e for e in out["fp64"]["series"]}
    for mode in ("mixed", "fp32"):
        cmp = []
        for e in out[mode]["series"]:
            f = ref.get(e["step"])
            if f is None:
                continue
            cmp.append({"step": e["step"], "t_rel": e["t"] / f["t"] - 1.0,
                        "T_rise_rel": (e["mean_T_rise_K"] - f["mean_T_rise_K"]) / abs(f["mean_T_rise_K"]),
                        "torque_rel": (e["disk_torque_mean_Nm"] - f["disk_torque_mean_Nm"]) / abs(f["disk_torque_mean_Nm"]),
                        "mass_proxy_drift_diff": e["mass_proxy_drift"] - f["mass_proxy_drift"]})
        out[mode]["vs_fp64"] = cmp
    if final.get("mixed") is not None and final.get("fp64") is not None:
        umax = c.meta["umax"]
        g, f = final["mixed"], final["fp64"]
        out["mixed"]["final_field_rms_vs_fp64"] = {
            "v_over_umax": float(np.sqrt(np.mean(np.sum((g["v"] - f["v"]) ** 2, axis=1))) / umax),
            "rho_over_rho0": float(np.sqrt(np.mean((g["rho"] - f["rho"]) ** 2)) / c.params["rho0"])}
    print(json.dumps({"metric": "precision study: drift vs FP64 GPU reference", "config": {
        "workload": f"churning tank dp={args.ps_dp * 1e3:.3f} mm, disk 450 rad/s, {args.ps_steps} steps",
        "n_fluid": c.nf, "n_solid": c.ns}, "modes": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--timed-steps", type=int, default=20, help="steps of the per-kernel event-timed pass")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64", "fp32"])
    ap.add_argument("--dp", type=float, default=1.5e-3, help="particle spacing of the gearbox proxy")
    ap.add_argument("--workload", default="gearbox", choices=["gearbox", "full", "fine"],
                    help="gearbox: the 1.5 mm proxy at 300 rad/s (default); full: the 1 mm proxy at 600 rad/s; "
                         "fine: the full proxy at dp = 0.8 mm (about 5.9 M particles)")
    ap.add_argument("--viscous-heating", action="store_true",
                    help="add the viscous dissipation heating of eq. 23 (off in the paper's model)")
    ap.add_argument("--materials", action="store_true",
                    help="two fluid materials (eq. 22 with k_i, cp_i), split at the box's mid-plane x")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--calib-copy", action="store_true", help="run one 1 GiB device copy (counter calibration)")
    ap.add_argument("--serve", action="store_true", help="serving sweep instead of the single-solve bench")
    ap.add_argument("--serve-n", type=int, default=64)
    ap.add_argument("--serve-steps", type=int, default=500)
    ap.add_argument("--serve-scale", type=float, default=1.0, help="multiplies every request's particle count")
    ap.add_argument("--serve-budget-gb", type=float, default=24.0)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-seeds", type=int, default=1, help="arrival seeds (64, 65, ...)")
    ap.add_argument("--no-serving", action="store_true", help="leave the reduced serving sweep out of the line")
    ap.add_argument("--quick-serve-n", type=int, default=32)
    ap.add_argument("--quick-serve-steps", type=int, default=300)
    ap.add_argument("--quick-serve-scale", type=float, default=0.5)
    ap.add_argument("--quick-serve-seeds", type=int, default=3)
    ap.add_argument("--spin-up", type=int, default=100,
                    help="untimed steps before the warm-up, past the acoustic transient of the gears' "
                         "impulsive start (about 60 steps)")
    ap.add_argument("--cpu-one-thread-steps", type=int, default=1,
                    help="advection steps of the one-thread oracle sample (0: none)")
    ap.add_argument("--relax", action="store_true",
                    help="particle relaxation of the 40-tooth gear body instead of the solver bench")
    ap.add_argument("--relax-iters", type=int, default=50)
    ap.add_argument("--contact", action="store_true",
                    help="contact factor (eq. 24) of the gearbox proxy's solid particles instead of the solver bench")
    ap.add_argument("--contact-calls", type=int, default=20)
    ap.add_argument("--precision-study", action="store_true",
                    help="churning tank in fp32 / mixed / fp64: drift of the conserved quantities")
    ap.add_argument("--ps-steps", type=int, default=100000)
    ap.add_argument("--ps-dp", type=float, default=0.788e-3)
    ap.add_argument("--ps-ckpt", type=int, default=5000, help="steps between precision-study checkpoints")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py runs on one GPU only: every box here has a single MI355X and the path is "
              "measured on one GPU's share; see the sharding design for more GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_09904_amd import cases, sph

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        return

    if args.serve:
        serve_bench(args)
        return
    if args.precision_study:
        precision_study(args)
        return
    if args.relax:
        relax_bench(args)
        return
    if args.contact:
        contact_bench(args)
        return

    t0 = time.perf_counter()
    if args.workload in ("full", "fine"):
        # the full-size proxy: 40-tooth gear at 600 rad/s, 50 mm immersion, nu = 2.2e-4
        om, imm, nu, dp = 600.0, 0.050, 2.2e-4, (1e-3 if args.workload == "full" else 0.8e-3)
    else:
        om, imm, nu, dp = 300.0, 0.030, 1e-4, args.dp
    case = cases.gearbox(seed=0, dp=dp, omega_big=om, immersion=imm, nu=nu)
    if args.viscous_heating:
        case.params["viscous_heating"] = 1
    if args.materials:
        case.params["materials"] = [(case.params["k_f"], case.params["cp_f"]), (0.45, 1300.0)]
        case.material = (case.xf[:, 0] > 0.5 * (case.xf[:, 0].min() + case.xf[:, 0].max())).astype(np.int32)
    log(f"case: nf={case.nf} ns={case.ns} generated in {time.perf_counter() - t0:.1f} s")
    s = sph.Solver(case, precision=args.precision)
    log("initialised")
    # untimed spin-up past the impulsive start (the acoustic transient of the
    # sudden start crosses the box a few times at c0 within about 60 steps)
    if args.spin_up:
        s.step(args.spin_up)
        s.reduce()
        log(f"spin-up: {args.spin_up} steps")
    s.step(args.warmup)
    r0 = s.reduce()
    pf0, ps0 = pair_counts(s, case.nf)

    # timed region 1: captured graph per advection step
    torch.cuda.synchronize()
    s.stream.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    r = s.reduce()
    s.stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    pf1, ps1 = pair_counts(s, case.nf)
    pairs = 0.5 * (pf0 + pf1) + 0.5 * (ps0 + ps1)
    n_ac = r["n_ac"]
    nsub = r["substeps"] - r0["substeps"]        # acoustic sub-steps in the timed region
    sweeps = (2 * args.steps + 2 * nsub) / args.steps
    ms_per_step = 1e3 * wall / args.steps
    value = pairs * (2 * args.steps + 2 * nsub) / wall
    log(f"graph: {ms_per_step:.3f} ms/step, n_ac={n_ac}, pairs/sweep={pairs:.3e}, {value:.3e} interactions/s")

    # timed region 2: the next steps launched eagerly with HIP events per kernel
    s.set_timing(True)
    t0 = time.perf_counter()
    nac_steps = []
    for _ in range(args.timed_steps):
        s.step(1)
        nac_steps.append(s.reduce()["n_ac"])
    wall2 = time.perf_counter() - t0
    kt = {k: s.timing(k) for k in sph.KERNELS}
    s.set_timing(False)
    # sub-step kernels are launched for the bound on n_ac; launches past a
    # step's n_ac exit at once and are dropped from the per-launch statistics
    # (sub-step 0's momentum runs inside the viscous/heat sweep: its own
    # launches cover sub-steps 1 ..)
    for k, first in (("momentum", 1), ("continuity", 0)):
        nl = len(kt[k]) // args.timed_steps
        kt[k + "_all"] = kt[k]
        kt[k] = np.concatenate([kt[k][q * nl: q * nl + max(0, nac_steps[q] - first)]
                                for q in range(args.timed_steps)])
    pf2, ps2 = pair_counts(s, case.nf)
    pbar = (pf2 + ps2) / case.nf
    per_step_kernel_ms = {k: float(kt[k + "_all" if k + "_all" in kt else k].sum() / args.timed_steps)
                          for k in sph.KERNELS if len(kt[k])}
    log("per-step kernel ms:", json.dumps({k: round(v, 4) for k, v in per_step_kernel_ms.items()}))
    nsr = distinct_wall_particles(s, case.nf)
    # lane gathers of neighbour records per launch (16-B records in mixed precision; the viscous/heat
    # sweep's fluid pairs: offsets, velocity state, the (T, Drho) record, and the material index with
    # two materials)
    gathers = {"momentum": 2 * (pf2 + ps2), "continuity": 2 * pf2 + 3 * ps2,
               "visc_heat": (4 if args.materials else 3) * pf2 + 3 * ps2, "sumw": 2 * (pf2 + ps2)}
    kern = {}
    for k in ("build", "sumw", "visc_heat", "momentum", "continuity"):
        if not len(kt[k]):
            continue      # momentum: every timed step had a single sub-step
        ms = float(np.mean(kt[k]))
        e = {"avg_launch_ms": round(ms, 5), "ms_per_step": round(per_step_kernel_ms[k], 4)}
        mb = model_bytes(k, case.nf, pbar)
        if mb is not None:
            e["model_bytes_per_launch"] = int(mb)
            e["model_GBs"] = round(mb / (ms * 1e-3) / 1e9, 1)
            e["model_frac"] = round(mb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        b = sweep_bytes(k, case.nf, nsr, pf2, ps2, args.precision)
        e["index_bytes_per_launch"] = int(b)
        e["index_GBs"] = round(b / (ms * 1e-3) / 1e9, 1)
        if k in gathers:
            e["lane_gathers_per_s"] = gathers[k] / (ms * 1e-3)
        kern[k] = e
    # the build is a search: 8 FP64 flops (three differences, three squares,
    # two sums) per candidate of the 27-cell stencil
    cand = build_candidates(s, case)
    b_flops = 8.0 * cand
    kern["build"]["candidates"] = cand
    kern["build"]["fp64_tflops"] = round(b_flops / (kern["build"]["avg_launch_ms"] * 1e-3) / 1e12, 3)
    kern["build"]["fp64_frac"] = round(kern["build"]["fp64_tflops"] / FP64_PEAK_TFLOPS, 4)
    # the dominant kernel: the largest share of the step's device time among
    # the pair sweeps of the byte model
    dom = max((k for k in kern if "model_bytes_per_launch" in kern[k]), key=lambda k: kern[k]["ms_per_step"])
    avg_ms = kern[dom]["avg_launch_ms"]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        ent = tr.get(dom, {})
        # counters are per launch of one workload: they stand only for that one
        wl = {"n_fluid": case.nf, "n_solid": case.ns, "viscous_heating": int(args.viscous_heating),
              "n_materials": 2 if args.materials else 1}
        if (tr.get("kernel_sha") == kernel_hash() and tr.get("precision") == args.precision
                and tr.get("workload") == wl):
            traffic = ent.get("bytes_per_launch")
    achieved = kern[dom]["model_GBs"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "k_" + dom,
                "bytes_per_launch": kern[dom]["model_bytes_per_launch"], "avg_launch_ms": avg_ms,
                "basis": f"pair-record byte model: {case.nf} fluid particles x ({MODEL_TEXT[dom].format(p=pbar)}) "
                         f"per launch, {pbar:.2f} mean ordered pairs per fluid particle",
                "index_design": {"bytes_per_launch": kern[dom]["index_bytes_per_launch"],
                                 "GBs": kern[dom]["index_GBs"],
                                 "basis": "bytes this design streams: 4-B row indices, each particle and wall "
                                          "record once"},
                "lane_gathers_per_s": kern[dom].get("lane_gathers_per_s")}
    sweep_lat = {k: {"p50_ms": round(pct(kt[k], 50), 5), "p99_ms": round(pct(kt[k], 99), 5), "n": len(kt[k])}
                 for k in ("build", "visc_heat", "momentum", "continuity") if len(kt[k])}
    s.close()

    serving = None
    if not args.no_serving:
        log("serving: reduced parameter sweep, batched vs one at a time")
        serving = serve_quick(args)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        cpu = cpu_baseline(case, args.cpu_steps)
        log(f"cpu baseline: {cpu['value']:.3e} interactions/s on {cpu['cores']} threads")
        if args.cpu_one_thread_steps:
            one = cpu_baseline(case, args.cpu_one_thread_steps, threads=1)
            cpu["one_thread"] = {"value": one["value"], "steps_per_s": one["steps_per_s"], "sample": one["sample"]}
            log(f"cpu baseline, one thread: {one['value']:.3e} interactions/s")

    hist = {str(k): int(v) for k, v in zip(*np.unique(nac_steps, return_counts=True))}
    out = {
        "metric": "particle-interactions/s & steps/s at 1M particles; p50/p99 sweep latency",
        "value": value,
        "unit": "particle-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "steps_per_s": 1e3 / ms_per_step,
        "acoustic_substeps_per_s": nsub / wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f32+f64", "fp64": "f64", "fp32": "f32"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"gearbox proxy dp={dp * 1e3:.2f} mm, two toothed disks 20/40 teeth at "
                               f"-{2 * om:.0f}/{om:.0f} rad/s, {imm * 1e3:.0f} mm immersion, nu={nu:g}"
                               + (", viscous dissipation heating" if args.viscous_heating else "")
                               + (", two fluid materials" if args.materials else ""),
                   "n_fluid": case.nf, "n_solid": case.ns, "spin_up_steps": args.spin_up,
                   "pairs_per_sweep": int(pairs), "mean_pairs_per_fluid_particle": round(pbar, 3),
                   "pair_sweeps_per_step": round(sweeps, 3), "precision": args.precision,
                   "parallelism": "single GPU"},
        "substeps": {"timed_mean_n_ac": round(nsub / args.steps, 3), "n_ac_first": r0["n_ac"], "n_ac_last": n_ac,
                     "event_timed_n_ac_histogram": hist},
        "sweep_latency": sweep_lat,
        "event_timed": {"steps": args.timed_steps, "ms_per_step": 1e3 * wall2 / args.timed_steps,
                        "kernel_ms_per_step": {k: round(v, 4) for k, v in per_step_kernel_ms.items()},
                        "kernels": kern, "wall_particles_in_rows": nsr},
        "roofline": roofline,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
