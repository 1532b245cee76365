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
GATHER_PEAK = 256 * 2.4e9
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
        # vr, offsets, T, counts read; ah written; wall offsets, velocities, lever arms
        return nf * (v4 + v4 + pb + cnt + v4) + rows + nsr * 3 * v4
    if kernel == "build":
        # anchors read; offsets and counts written; rows written (the particle-major staging is
        # read back from cache); wall positions
        return nf * (4 * pb + v4 + cnt) + rows + nsr * 4 * pb
    if kernel == "sumw":
        # anchors, counts read; sum W written; vr read and written; rows read; wall positions
        return nf * (4 * pb + cnt + 8 + 2 * v4) + rows + nsr * 4 * pb
    raise KeyError(kernel)


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


def cpu_baseline(case, steps=6):
    """The FP64 oracle on the host cores, on a bounded sample of the same workload."""
    from oracle import oracle as O
    O.build(force=False)
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
    cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    return {"value": (pf + ps) * sweeps / dt, "unit": "particle-interactions/s", "cores": cores,
            "kind": "oracle", "steps_per_s": steps / dt,
            "sample": f"{steps} advection steps of the full gearbox proxy (dp 1.5 mm, {case.nf} fluid + {case.ns} "
                      f"solid particles) from the initial state, FP64 C/OpenMP oracle, {dt:.1f} s"}


def serve_bench(args):
    """Parameter-sweep serving: continuous batching vs one solve at a time.

    Requests: shaft speed U(150, 600) rad/s, immersion U(20, 60) mm, nu
    U(0.5, 3)e-4, fluid count log-uniform 50k-2M, `serve_steps` advection steps
    each.  Each request's service time alone is measured first (one slot);
    arrivals are Poisson with rate 0.85 / mean service time; the
    one-at-a-time server's latencies follow exactly from the measured service
    times (FIFO); the batched server is run live.
    """
    import torch
    from paper_2512_09904_amd import serve, sph
    budget = int(args.serve_budget_gb * (1 << 30))
    t0 = time.perf_counter()
    reqs = serve.sweep_requests(n=args.serve_n, seed=64, steps=args.serve_steps, scale=args.serve_scale)
    log(f"generated {len(reqs)} requests in {time.perf_counter() - t0:.1f} s; "
        f"fluid {sum(r.case.nf for r in reqs)} total")
    # service time of each request alone
    svc = []
    for r in reqs:
        pool = sph.Pool(budget, max_slots=1)
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
    for seed in range(64, 64 + args.serve_seeds):
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
        for r, a in zip(reqs, arr):
            r.arrival = float(a)
            r.admitted = r.finished = r.report = None
        srv = serve.Server(budget, max_slots=args.serve_slots)
        a = time.perf_counter()
        ndone = [0]

        def progress(r, nact, nq, npend):
            ndone[0] += 1
            if ndone[0] % 8 == 0:
                log(f"batched: {ndone[0]} done, {nact} active, {nq} queued, {npend} not arrived")

        srv.run(reqs, progress=progress)
        wall = time.perf_counter() - a
        summ = serve.summarize(reqs, wall)
        same = all(np.array_equal(r.report["bodies"][1]["torque_axis"], r.alone["bodies"][1]["torque_axis"]) and
                   r.report["heat_total"] == r.alone["heat_total"] for r in reqs)
        results.append(dict(seed=seed, rate_per_s=rate, batched=summ, peak_slots=srv.peak_active,
                            peak_gb=srv.peak_bytes / (1 << 30), results_equal_alone=bool(same),
                            one_at_a_time=dict(p50_s=float(np.percentile(lat1, 50)),
                                               p95_s=float(np.percentile(lat1, 95)),
                                               p99_s=float(np.percentile(lat1, 99)),
                                               wall_s=float(fin.max()),
                                               particle_steps_per_s=float(sum(r.case.nf * r.steps for r in reqs) / fin.max()))))
        srv.close()
        log(json.dumps(results[-1]))
    b = results[0]["batched"]
    out = {"metric": "serving sweep: p50/p99 time-to-result and throughput, batched vs one at a time",
           "value": b["particle_steps_per_s"], "unit": "fluid particle-steps/s", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic", "dtype": "f32+f64",
           "config": {"workload": f"{len(reqs)} serving-tank requests, {args.serve_steps} steps each, Poisson "
                                  f"arrivals at 0.85/mean service, budget {args.serve_budget_gb} GB, "
                                  f"{args.serve_slots} slots, particle scale {args.serve_scale}"},
           "mean_service_alone_s": sbar, "seeds": results}
    print(json.dumps(out), flush=True)


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

    # timed region 2: the same steps launched eagerly with HIP events per kernel
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
    for k in ("momentum", "continuity"):
        nl = len(kt[k]) // args.timed_steps
        kt[k + "_all"] = kt[k]
        kt[k] = np.concatenate([kt[k][q * nl: q * nl + nac_steps[q]] for q in range(args.timed_steps)])
    pf2, ps2 = pair_counts(s, case.nf)
    per_step_kernel_ms = {k: float(kt[k + "_all" if k + "_all" in kt else k].sum() / args.timed_steps)
                          for k in sph.KERNELS if len(kt[k])}
    log("per-step kernel ms:", json.dumps({k: round(v, 4) for k, v in per_step_kernel_ms.items()}))
    nsr = distinct_wall_particles(s, case.nf)
    kern = {}
    for k in ("build", "sumw", "visc_heat", "momentum", "continuity"):
        b = sweep_bytes(k, case.nf, nsr, pf2, ps2, args.precision)
        ms = float(np.mean(kt[k]))
        kern[k] = {"bytes_per_launch": int(b), "avg_launch_ms": round(ms, 5),
                   "achieved_GBs": round(b / (ms * 1e-3) / 1e9, 1),
                   "frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "ms_per_step": round(per_step_kernel_ms[k], 4)}
    # the build is a search, bound by vector FP64 arithmetic: its algorithmic
    # work is 8 FP64 flops (three differences, three squares, two sums) per
    # candidate of the 27-cell stencil
    cand = build_candidates(s, case)
    b_flops = 8.0 * cand
    kern["build"]["candidates"] = cand
    kern["build"]["fp64_tflops"] = round(b_flops / (kern["build"]["avg_launch_ms"] * 1e-3) / 1e12, 3)
    kern["build"]["fp64_frac"] = round(kern["build"]["fp64_tflops"] / FP64_PEAK_TFLOPS, 4)
    # the dominant kernel: the largest share of the step's device time
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
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
    if dom == "build":
        roofline = {"bound": "alu", "achieved": kern["build"]["fp64_tflops"], "peak": FP64_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": kern["build"]["fp64_frac"], "traffic": traffic, "kernel": "k_build",
                    "flops_per_launch": b_flops, "avg_launch_ms": avg_ms}
    else:
        achieved = kern[dom]["achieved_GBs"]
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": "k_" + dom,
                    "bytes_per_launch": int(kern[dom]["bytes_per_launch"]), "avg_launch_ms": avg_ms}
        # the sweeps are limited by scattered 16-byte gathers, which the vector
        # memory unit serves at about one lane per clock per CU
        gathers = {"momentum": 2 * (pf2 + ps2), "continuity": 2 * pf2 + 3 * ps2,
                   "visc_heat": 3 * (pf2 + ps2), "sumw": 2 * (pf2 + ps2)}.get(dom)
        if gathers:
            rate = gathers / (avg_ms * 1e-3)
            roofline["gather_rate"] = {"achieved": rate, "peak": GATHER_PEAK, "unit": "lane gathers/s",
                                       "frac": round(rate / GATHER_PEAK, 4), "gathers_per_launch": int(gathers),
                                       "peak_basis": "one scattered lane per clock per CU, 256 CUs at 2.4 GHz "
                                                     "(texture-addresser and L1 counters)"}
    sweep_lat = {k: {"p50_ms": round(pct(kt[k], 50), 5), "p99_ms": round(pct(kt[k], 99), 5), "n": len(kt[k])}
                 for k in ("build", "visc_heat", "momentum", "continuity") if len(kt[k])}

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        cpu = cpu_baseline(case, args.cpu_steps)
        log(f"cpu baseline: {cpu['value']:.3e} interactions/s on {cpu['cores']} threads")

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
                   "n_fluid": case.nf, "n_solid": case.ns, "n_ac_last": n_ac, "pairs_per_sweep": int(pairs),
                   "pair_sweeps_per_step": round(sweeps, 3), "precision": args.precision, "parallelism": "single GPU"},
        "sweep_latency": sweep_lat,
        "event_timed": {"steps": args.timed_steps, "ms_per_step": 1e3 * wall2 / args.timed_steps,
                        "kernel_ms_per_step": {k: round(v, 4) for k, v in per_step_kernel_ms.items()},
                        "kernels": kern, "wall_particles_in_rows": nsr},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
