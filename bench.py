#!/usr/bin/env python3
"""Benchmark of one mechanics iteration at scale on one MI355X.

Workload (default): plain mechanics, 1e8 agents uniform in a cube at 1 agent
per 1000 um^3, diameters U[10, 15) um, box length 15 um, dt 0.01, k = 2,
gamma = 1, adherence 1.8, mass 0.1, cap 3 um, Morton re-sort every 10
iterations; FP32 forces, FP64 positions.  ``--workload relaxed`` runs the
pre-relaxed lattice (most agents static, static skip on); ``spheroid`` grows
one tumour spheroid from 1,000 cells to about 5e6; ``sweep`` and
``surrogate`` time the batched parameter sweep and the surrogate screening;
``apoptosis`` adds the Brownian step and apoptosis of Algorithm 2; ``sir``
runs Table 4.5's large-scale measles epidemic (1.01e7 persons, 1,000
iterations); ``soma`` runs Table 5.1's cell clustering (2e6 cells, two
substances diffusing on 300^3 points).

A step is one iteration of the whole hot path (grid build, force sweep,
displacement, static flags, re-sort when due).  Prints one JSON line with the
throughput (agent updates per second), the roofline of the force sweep (its
duration measured with HIP events on the stream it runs on, during the timed
region) and the FP64 oracle timed on this host's cores on a bounded sample.
"""
import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of the force sweep per agent: FP64 position read and
# write (48), own radius (diameter, 8), box key and arrival rank (8), flags
# and non-zero-force count read/write (3), the agent's FP32 payload read once
# as a neighbour (16); plus 4 bytes per grid box of slot starts.
SWEEP_BYTES_PER_AGENT = 48 + 8 + 8 + 3 + 16
SWEEP_BYTES_PER_BOX = 4
PMC_FILE = os.path.join(ROOT, "profiles", "sweep_c1_pmc.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    with open(os.path.join(ROOT, "paper_2503_10796_amd", "csrc", "abm_mech.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(n_agents, workload):
    """HBM bytes per sweep launch from the committed rocprofv3 counter runs,
    or None when they are missing or the kernel changed since."""
    if not os.path.exists(PMC_FILE):
        return None
    with open(PMC_FILE) as f:
        pmc = json.load(f)
    if pmc.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    if pmc.get("agents") != n_agents or pmc.get("workload") != workload:
        return None
    return pmc.get("hbm_bytes_per_launch")


def oracle_sample(workload, n, iters):
    """Time the FP64 oracle for `iters` iterations (after one untimed one) on
    `n` agents of the mechanics workload; returns (agents, seconds)."""
    sys.path.insert(0, ROOT)
    from oracle import sim as osim
    from paper_2503_10796_amd import inputs
    if workload == "uniform":
        pos, diam = inputs.at_density(n, seed=1)
        detect = False
    else:
        side = round(n ** (1.0 / 3.0))
        pos, diam = inputs.relaxed_lattice(side, seed=2)
        detect = True
    o = osim.OracleSim(pos, diam, osim.make_params(box_len=15.0, detect_static=detect))
    o.step(1)  # first iteration untimed (initialisation excluded)
    t0 = time.perf_counter()
    o.step(iters)
    return pos.shape[0], time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args):
    """The FP64 oracle as it stands on a bounded sample of the same workload:
    with the host's OpenMP threads, and single-threaded (a child process with
    one OpenMP thread) on a smaller sample."""
    n, dt = oracle_sample(args.workload, args.cpu_sample_agents, args.cpu_sample_iters)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": n * args.cpu_sample_iters / dt, "unit": "agent updates/s", "cores": threads,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{n} agents of the same workload (same density and diameters), {args.cpu_sample_iters} "
                     f"iterations after one untimed iteration, FP64, OpenMP over agents, {dt:.1f} s"}
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-sample", args.workload,
                        str(args.cpu_single_agents), str(args.cpu_single_iters)],
                       env=env, capture_output=True, text=True, timeout=600)
    if r.returncode == 0:
        n1, dt1 = json.loads(r.stdout.strip().splitlines()[-1])
        out["single_thread"] = {"value": n1 * args.cpu_single_iters / dt1, "unit": "agent updates/s", "cores": 1,
                                "sample": f"{n1} agents, {args.cpu_single_iters} iterations after one untimed "
                                          f"iteration, one OpenMP thread, {dt1:.1f} s"}
    else:
        out["single_thread"] = None
        log(f"[bench] single-thread oracle sample failed: {r.stderr[-500:]}")
    return out


def _counter_per_dispatch(path, kernel_substr, counter):
    """Mean over dispatches of a kernel of one counter (summed over its
    hardware instances) from a rocprofv3 csv counter file."""
    import csv
    per = {}
    for r in csv.DictReader(open(path)):
        if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter:
            per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return sum(per.values()) / len(per), len(per)


def pmc_summary(args):
    """HBM bytes of one force-sweep launch from the byte counters, each scaled
    by what the same counter reads for a plain copy of known size."""
    fetch, write, cfetch, cwrite = args.pmc_summary
    f_kib, nf = _counter_per_dispatch(fetch, "k_sweep<", "FETCH_SIZE")
    w_kib, nw = _counter_per_dispatch(write, "k_sweep<", "WRITE_SIZE")
    cf_kib, _ = _counter_per_dispatch(cfetch, "copyBuffer", "FETCH_SIZE")
    cw_kib, _ = _counter_per_dispatch(cwrite, "copyBuffer", "WRITE_SIZE")
    copy_bytes = 2 ** 31
    f_scale = copy_bytes / (cf_kib * 1024.0)
    w_scale = copy_bytes / (cw_kib * 1024.0)
    read_b = f_kib * 1024.0 * f_scale
    write_b = w_kib * 1024.0 * w_scale
    out = {"kernel": "k_sweep", "workload": args.workload, "agents": args.agents,
           "kernel_source_sha256_16": kernel_source_hash(),
           "fetch_kib_per_launch": f_kib, "write_kib_per_launch": w_kib, "dispatches": [nf, nw],
           "copy_fetch_kib": cf_kib, "copy_write_kib": cw_kib, "fetch_scale": f_scale, "write_scale": w_scale,
           "hbm_read_bytes_per_launch": read_b, "hbm_write_bytes_per_launch": write_b,
           "hbm_bytes_per_launch": read_b + write_b}
    with open(PMC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


def copy_calibration(torch, steps):
    """A plain copy of known size: the HBM byte counters of one such launch,
    divided by the bytes it must move (2 GiB read, 2 GiB written), give the
    scale factor for the counters of the other kernels."""
    n = 2 ** 31 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": steps}), flush=True)


def bench_sweep(args):
    """Batched parameter sweep (one graph launch per iteration for all
    simulations) against the per-simulation path on the same simulations."""
    import numpy as np
    import torch
    from paper_2503_10796_amd import sweep
    cfg = sweep.SweepConfig(args.sims, seed=4, iters=args.sweep_iters)
    t_gen = time.perf_counter()
    counts = np.array([cfg.counts(s, *cfg.state(s)[2:4]) for s in range(cfg.n_sims)])
    updates = float(counts[:, :cfg.iters].sum())
    log(f"[bench] sweep inputs and exact agent counts in {time.perf_counter() - t_gen:.1f} s; "
        f"{int(counts[:, 0].sum())} agents at the start, {int(counts[:, -1].sum())} at the end")
    _, t_batch, n_end, sched = sweep.run_batched(cfg, record=False, tune=True, log=log)
    assert np.array_equal(n_end, counts[:, -1].astype(np.int64)), "agent counts differ from the lineage count"
    if args.batched_only:
        t_single = float("nan")
    else:
        secs = sweep.run_per_sim(cfg, list(range(cfg.n_sims)))
        t_single = float(secs.sum())
        log(f"[bench] per-simulation path: {t_single:.3f} s for {cfg.n_sims} simulations")
    out = {
        "metric": "batched parameter sweep: agent updates/s, speedup over the per-simulation path",
        "value": updates / t_batch, "unit": "agent updates/s", "n_gpus": 1, "steps": cfg.iters, "warmup": 1,
        "ms_per_step": t_batch / cfg.iters * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"tumour-spheroid sweep: {cfg.n_sims} simulations, Latin hypercube seed 4 over growth "
                               f"scale [0.5,1.5], division diameter [6,18] um, adherence [0.9,2.7]; initial counts "
                               f"log-uniform [1e3,5e4]; {cfg.iters} iterations",
                   "agents_start": int(counts[:, 0].sum()), "agents_end": int(counts[:, -1].sum()),
                   "schedule": sched},
        "batched_s": t_batch, "per_simulation_s": None if args.batched_only else t_single,
        "speedup_vs_per_simulation": None if args.batched_only else t_single / t_batch,
    }
    if not args.no_cpu_baseline and not args.batched_only:
        log("[bench] timing the oracle on the host")
        out["cpu_baseline"] = sweep_cpu_baseline(args, cfg)
    print(json.dumps(out), flush=True)


def sweep_cpu_baseline(args, cfg):
    """The oracle on a bounded sample of the sweep: its first simulations,
    one after another, over the first iterations (the oracle has no batching:
    simulations are independent)."""
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import sim as osim
    from paper_2503_10796_amd import inputs
    sims, iters = list(range(args.sweep_cpu_sims)), args.sweep_cpu_iters
    updates, dt = 0.0, 0.0
    for s in sims:
        pos, diam, vol, growth = cfg.state(s)
        counts = cfg.counts(s, vol, growth)
        o = osim.OracleSim(pos, diam, osim.make_params(box_len=0.0, div_vol=inputs.division_volume(float(cfg.d_div[s])),
                                                       adherence=float(cfg.adherence[s]), detect_static=True,
                                                       seed=cfg.seed, sim_id=s),
                           vol=vol, growth=growth, cap=int(counts[iters]) + 16)
        t0 = time.perf_counter()
        o.step(iters)
        dt += time.perf_counter() - t0
        updates += float(np.asarray(counts[:iters]).sum())
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": updates / dt, "unit": "agent updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"simulations {sims[0]}..{sims[-1]} of the same sweep, one after another, over their first "
                      f"{iters} iterations ({updates:.3g} updates), FP64, OpenMP over agents, {dt:.1f} s"}


def lineage_counts(vol, growth, vdiv, iters):
    """Agent count at every iteration 0..iters.  Growth and division do not
    depend on positions (a cell grows by its rate below the division volume,
    else splits into two halves with the same rate), so the count follows from
    the volumes alone, with the same FP64 operations as the step."""
    V = np.array(vol, dtype=np.float64)
    m = np.ones_like(V)
    out = [float(m.sum())]
    for _ in range(iters):
        div = V >= vdiv
        V = np.where(div, 0.5 * V, V + growth)
        m = np.where(div, 2.0 * m, m)
        out.append(float(m.sum()))
    return np.array(out)


def bench_spheroid(args):
    """Tumour-spheroid growth at scale: 1,000 cells in a 50 um ball grown to
    about 5e6 agents.  The growth rates are the lognormal draws of the
    spheroid recipe times a scale factor chosen so that the lineage count
    reaches about 5e6 at the last iteration (the literal rates give about
    1.35e3 agents after 600 iterations)."""
    import torch
    from paper_2503_10796_amd import abm, inputs
    abm.lib()
    S, iters = args.spheroid_scale, args.spheroid_iters
    pos, diam, vol, growth = inputs.spheroid(1000, seed=3, growth_scale=S)
    vdiv = inputs.division_volume(12.0)
    counts = lineage_counts(vol, growth, vdiv, iters)
    cap = int(1.05 * counts[-1]) + 1024
    p = abm.params(box_len=0.0, div_vol=vdiv, seed=3, resort_every=args.resort_every, detect_static=False)
    pop = abm.Population(p, pos, diam, vol=vol, growth=growth, capacity=cap)
    log(f"[bench] spheroid: growth scale {S}, {iters} iterations, lineage count {int(counts[-1])}, capacity {cap}")
    torch.cuda.synchronize()
    chunk = 50
    marks = []
    t0 = time.perf_counter()
    done = 0
    while done < iters:
        k = min(chunk, iters - done)
        pop.step(k)
        torch.cuda.synchronize()
        done += k
        marks.append((done, time.perf_counter() - t0, int(pop.num_agents()[0])))
        log(f"[bench] iteration {done}: {marks[-1][2]} agents, {marks[-1][1]:.2f} s")
    elapsed = marks[-1][1]
    n_end = marks[-1][2]
    assert n_end == int(counts[-1]), f"agent count {n_end} differs from the lineage count {int(counts[-1])}"
    updates = float(counts[:iters].sum())
    c, rg, rm, _ = pop.stats(hist_rmax=400.0)
    last_ms = (marks[-1][1] - marks[-2][1]) / (marks[-1][0] - marks[-2][0]) * 1e3 if len(marks) > 1 else None
    out = {
        "metric": "tumour-spheroid growth: agent updates/s over the whole run",
        "value": updates / elapsed, "unit": "agent updates/s", "n_gpus": 1, "steps": iters, "warmup": 0,
        "ms_per_step": elapsed / iters * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"tumour spheroid: 1000 cells in a 50 um ball (seed 3), d = 8 um, lognormal growth "
                               f"(mean 1 um^3/step, log-sigma 0.2) times {S}, division at 12 um, box = largest "
                               f"diameter, Morton re-sort every {args.resort_every} iterations, {iters} iterations",
                   "growth_scale": S, "agents_start": 1000, "agents_end": n_end},
        "seconds": elapsed,
        "ms_per_step_last_chunk": last_ms,
        "progress": [{"iteration": it, "seconds": t, "agents": n} for it, t, n in marks],
        "r_gyr_um_end": float(rg[0]), "r_max_um_end": float(rm[0]),
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        out["cpu_baseline"] = spheroid_cpu_baseline(args)
    print(json.dumps(out), flush=True)


def spheroid_cpu_baseline(args):
    """The oracle on the same spheroid (same seed and growth scale) over its
    first iterations, while the population is small enough to finish in
    seconds."""
    sys.path.insert(0, ROOT)
    from oracle import sim as osim
    from paper_2503_10796_amd import inputs
    S, iters = args.spheroid_scale, args.spheroid_cpu_iters
    pos, diam, vol, growth = inputs.spheroid(1000, seed=3, growth_scale=S)
    vdiv = inputs.division_volume(12.0)
    counts = lineage_counts(vol, growth, vdiv, iters)
    o = osim.OracleSim(pos, diam, osim.make_params(box_len=0.0, div_vol=vdiv, seed=3), vol=vol, growth=growth,
                       cap=int(counts[-1]) + 16)
    t0 = time.perf_counter()
    o.step(iters)
    dt = time.perf_counter() - t0
    updates = float(counts[:iters].sum())
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": updates / dt, "unit": "agent updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"the same spheroid over its first {iters} iterations (1000 -> {int(counts[-1])} agents, "
                      f"{updates:.3g} updates), FP64, OpenMP over agents, {dt:.1f} s"}


def bench_apoptosis(args):
    """Algorithm 2 cell behaviour at scale: the uniform mechanics population
    (1 agent per 1000 um^3, diameters U[10,15) um, box 15 um) with the
    Table 4.2 Brownian step (0.005 um) and apoptosis (minimum age 87, death
    probability 0.033), initial ages uniform in [0, 100): every iteration
    removes cells, which the removal kernels compact out of the state."""
    import numpy as np
    import torch
    from paper_2503_10796_amd import abm, inputs
    abm.lib()
    n = args.agents
    pos, diam = inputs.at_density(n, seed=1)
    age = np.random.default_rng(7).integers(0, 100, size=n).astype(np.int32)
    side = inputs.cube_side(n)
    box_cap = int(1.1 * (side / 15.0 + 4.0) ** 3) + 4096
    p = abm.params(box_len=15.0, resort_every=args.resort_every, seed=9, brownian_rate=0.005, death_prob=0.033,
                   min_age=87)
    pop = abm.Population(p, pos, diam, capacity=n, box_capacity=box_cap)
    del pos, diam
    pop.restore(age=age)
    pop.set_sweep_grid(SWEEP_GRID["uniform"])
    torch.cuda.synchronize()
    pop.step(args.warmup)
    torch.cuda.synchronize()
    n0 = int(pop.num_agents()[0])
    t0 = time.perf_counter()
    pop.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n1 = int(pop.num_agents()[0])
    updates = float(n0 + n1) / 2.0 * args.steps
    log(f"[bench] apoptosis: {n0} -> {n1} agents over {args.steps} timed iterations in {elapsed:.3f} s")
    out = {
        "metric": "Algorithm 2 cell behaviour with removals: agent updates/s",
        "value": updates / elapsed, "unit": "agent updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{n} agents uniform in a {side:.1f} um cube (1 per 1000 um^3), diameters U[10,15) "
                               f"um, box 15 um, Brownian step 0.005 um, apoptosis from age 87 with probability "
                               f"0.033, initial ages U[0,100), Morton re-sort every {args.resort_every}",
                   "agents_start_timed": n0, "agents_end": n1,
                   "removed_per_iteration": (n0 - n1) / args.steps},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        out["cpu_baseline"] = apoptosis_cpu_baseline(args)
    print(json.dumps(out), flush=True)


def apoptosis_cpu_baseline(args):
    """The oracle on a bounded sample of the same workload: the uniform
    population at the same density with the same Brownian step, apoptosis
    parameters and age distribution."""
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import sim as osim
    from paper_2503_10796_amd import inputs
    n = args.cpu_sample_agents
    pos, diam = inputs.at_density(n, seed=1)
    age = np.random.default_rng(7).integers(0, 100, size=n).astype(np.int32)
    o = osim.OracleSim(pos, diam, osim.make_params(box_len=15.0, seed=9, brownian_rate=0.005, death_prob=0.033,
                                                   min_age=87), age=age)
    o.step(1)
    n0 = o.n
    t0 = time.perf_counter()
    o.step(args.cpu_sample_iters)
    dt = time.perf_counter() - t0
    updates = 0.5 * (n0 + o.n) * args.cpu_sample_iters
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": updates / dt, "unit": "agent updates/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n} agents of the same workload, {args.cpu_sample_iters} iterations after one untimed "
                      f"iteration ({n0} -> {o.n} agents), FP64, OpenMP over agents, {dt:.1f} s"}


# Algorithmic bytes of the SIR person kernel: per person, position 24, state
# 1 and uid 4 read, new position 24 and state 1 written in place; per person
# infected after the iteration (binned into the next index), box key 4 and
# rank 4 written and the box count's atomic read and write 8.
SIR_BEHAVE_BYTES = 29 + 25
SIR_BIN_BYTES = 8 + 8


def bench_sir(args):
    """Table 4.5's large-scale measles run: Table 4.3's measles model at
    `sir_scale` times the persons and the same density (default 5,000:
    1e7 susceptible + 1e5 infected in a 1,710 m torus), `steps` iterations
    (the thesis runs 1,000)."""
    import torch
    from paper_2503_10796_amd import abm, inputs
    abm.lib()
    cfg = inputs.scaled_sir(inputs.SIR_MEASLES, args.sir_scale)
    boundary = abm.CLOSED if args.sir_boundary == "closed" else abm.TOROIDAL
    t_gen = time.perf_counter()
    pos, st = inputs.sir_population(cfg["n_susceptible"], cfg["n_infected"], cfg["space"], seed=12)
    n = pos.shape[0]
    p = abm.sir_params(cfg["space"], cfg["radius"], cfg["infection_prob"], cfg["recovery_prob"], cfg["speed"],
                       boundary=boundary, seed=12)
    g = abm.Sir(p, pos, st, hist_cap=1024)
    del pos, st
    dims, box_len = g.grid()
    log(f"[bench] sir: {n} persons in a {cfg['space']:.1f} m cube, grid {dims}^3 boxes of {box_len:.3f} m, "
        f"set up in {time.perf_counter() - t_gen:.1f} s")
    g.set_timing(True)
    g.step(args.warmup)
    torch.cuda.synchronize()
    g.kernel_time()
    t0 = time.perf_counter()
    hist = g.step(args.steps, counts=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_ms, k_n = g.kernel_time()
    it, counts = g.counts()
    behave_bytes = (n * SIR_BEHAVE_BYTES * args.steps + SIR_BIN_BYTES * float(hist[:, 1].sum())) / max(args.steps, 1)
    log(f"[bench] sir: {args.steps} iterations in {elapsed:.3f} s; counts after iteration {it}: {counts.tolist()}")
    nbox = dims ** 3
    k_avg_s = k_ms / max(k_n, 1) / 1e3
    achieved = behave_bytes / k_avg_s / 1e9
    out = {
        "metric": "SIR epidemiology (Algorithms 3-5): person updates/s",
        "value": n * args.steps / elapsed, "unit": "person updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"measles SIR (Table 4.3) at {args.sir_scale} times the persons: "
                               f"{cfg['n_susceptible']} susceptible + {cfg['n_infected']} infected uniform in a "
                               f"{cfg['space']:.1f} m {args.sir_boundary} cube, radius {cfg['radius']} m, "
                               f"infection probability {cfg['infection_prob']}, recovery probability "
                               f"{cfg['recovery_prob']}, step {cfg['speed']} m; iterations "
                               f"{args.warmup}..{args.warmup + args.steps}",
                   "persons": n, "grid_boxes": nbox, "box_len_m": box_len,
                   "counts_end": counts.tolist()},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_sir_behave",
                     "kernel_ms": k_avg_s * 1e3, "algorithmic_bytes_per_launch": behave_bytes},
        "paper_context": "Table 4.5: 10,050,000 persons, 1,000 iterations in 59.19 s on 72 CPU cores "
                         "(1.70e8 person updates/s)",
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        out["cpu_baseline"] = sir_cpu_baseline(args)
    print(json.dumps(out), flush=True)


def sir_cpu_baseline(args):
    """The SIR oracle (brute-force neighbourhoods, O(N^2) per iteration) on
    the measles model at 10 times Table 4.3 (20,200 persons)."""
    sys.path.insert(0, ROOT)
    from oracle import sir as osir
    from paper_2503_10796_amd import inputs
    cfg = inputs.scaled_sir(inputs.SIR_MEASLES, args.sir_cpu_scale)
    pos, st = inputs.sir_population(cfg["n_susceptible"], cfg["n_infected"], cfg["space"], seed=12)
    op = osir.make_params(cfg["space"], cfg["radius"], cfg["infection_prob"], cfg["recovery_prob"], cfg["speed"],
                          boundary=osir.CLOSED if args.sir_boundary == "closed" else osir.TOROIDAL, seed=12)
    o = osir.OracleSIR(pos, st, op)
    t0 = time.perf_counter()
    o.step(args.sir_cpu_iters)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": pos.shape[0] * args.sir_cpu_iters / dt, "unit": "person updates/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"the same model at {args.sir_cpu_scale} times Table 4.3 ({pos.shape[0]} persons), the first "
                      f"{args.sir_cpu_iters} iterations, FP64, brute-force neighbourhoods (O(N^2): the rate falls "
                      f"with N), OpenMP over persons, {dt:.1f} s"}


# Algorithmic bytes of the diffusion kernel per grid point: the point read
# once and written once (its six neighbours come from registers, LDS or L2).
DIFFUSE_BYTES = 16


def bench_soma(args):
    """Table 5.1's cell clustering: 2e6 cells secreting and following two
    substances on 300^3 points each (5.4e7 diffusion volumes), `steps`
    iterations (the thesis runs 1,000)."""
    import torch
    from paper_2503_10796_amd import abm, inputs
    abm.lib()
    cfg = dict(inputs.SOMA_CELL_CLUSTERING)
    if args.soma_resolution:
        cfg["resolution"] = args.soma_resolution
    kw = {k: cfg[k] for k in ("lo", "space", "resolution", "n_substances", "diffusion", "decay", "dt", "secretion",
                              "gradient_weight")}
    t_gen = time.perf_counter()
    pos, t = inputs.soma_population(cfg, seed=7)
    g = abm.Soma(abm.soma_params(**kw), pos, t)
    n = pos.shape[0]
    del pos
    volumes = cfg["n_substances"] * cfg["resolution"] ** 3
    log(f"[bench] soma: {n} cells, {volumes} diffusion volumes, set up in {time.perf_counter() - t_gen:.1f} s")
    g.set_timing(True)
    g.step(args.warmup)
    torch.cuda.synchronize()
    g.kernel_time()
    t0 = time.perf_counter()
    g.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    k_ms, k_n = g.kernel_time()
    k_avg_s = k_ms / max(k_n, 1) / 1e3
    achieved = volumes * DIFFUSE_BYTES / k_avg_s / 1e9
    log(f"[bench] soma: {args.steps} iterations in {elapsed:.3f} s, diffusion kernel {k_avg_s * 1e3:.3f} ms")
    out = {
        "metric": "extracellular diffusion with soma clustering (Eq 4.3, Algorithms 6-7): diffusion volume updates/s",
        "value": volumes * args.steps / elapsed, "unit": "volume updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"cell clustering (Table 5.1): {n} cells of two types uniform in a "
                               f"{cfg['space']:.0f} um cube, two substances on {cfg['resolution']}^3 points, "
                               f"diffusion {cfg['diffusion']} um^2/step, decay {cfg['decay']}/step, secretion "
                               f"{cfg['secretion']}, gradient weight {cfg['gradient_weight']} um",
                   "cells": n, "volumes": volumes, "cell_updates_per_s": n * args.steps / elapsed},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "k_diffuse",
                     "kernel_ms": k_avg_s * 1e3, "algorithmic_bytes_per_launch": volumes * DIFFUSE_BYTES},
        "paper_context": "Table 4.5: soma clustering, 32,000 cells and 1,240,000 diffusion volumes, 6,000 "
                         "iterations in 12.91 s on 72 CPU cores (5.8e8 volume updates/s)",
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        out["cpu_baseline"] = soma_cpu_baseline(args)
    print(json.dumps(out), flush=True)


def soma_cpu_baseline(args):
    """The diffusion oracle on the same model at Table 4.5's soma clustering
    size (32,000 cells, two substances on 85^3 points)."""
    sys.path.insert(0, ROOT)
    from oracle import soma as osoma
    from paper_2503_10796_amd import inputs
    cfg = dict(inputs.SOMA_CELL_CLUSTERING)
    cfg.update(resolution=85, space=340.0, n_cells=32000)
    kw = {k: cfg[k] for k in ("lo", "space", "resolution", "n_substances", "diffusion", "decay", "dt", "secretion",
                              "gradient_weight")}
    pos, t = inputs.soma_population(cfg, seed=7)
    o = osoma.OracleSoma(pos, t, osoma.make_params(**kw))
    o.step(1)
    t0 = time.perf_counter()
    o.step(args.soma_cpu_iters)
    dt = time.perf_counter() - t0
    volumes = 2 * 85 ** 3
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": volumes * args.soma_cpu_iters / dt, "unit": "volume updates/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"the same model at Table 4.5's soma clustering size (32,000 cells, {volumes} volumes), "
                      f"{args.soma_cpu_iters} iterations after one untimed one, FP64, OpenMP over grid planes "
                      f"(cells serial), {dt:.1f} s"}


def bench_surrogate(args):
    """Surrogate screening: train on windows of a batched sweep, judge on the
    simulated histograms of held-out parameter sets, time the screening."""
    import numpy as np
    import torch
    from paper_2503_10796_amd import sweep, surrogate
    cfg = sweep.SweepConfig(args.sims, seed=4, iters=args.sweep_iters)
    hist, t_train_sim, _, _ = sweep.run_batched(cfg, record=True, tune=False, log=log)
    x, y = surrogate.windows(cfg, hist, 20000, seed=6, t_max=cfg.iters - surrogate.HORIZON, early=args.early_windows)
    model, t_train = surrogate.train(x, y, steps=args.train_steps, log=log)
    log(f"[bench] trained {args.train_steps} steps in {t_train:.2f} s")
    held = sweep.SweepConfig(2 * args.sims, seed=5, iters=cfg.iters)
    parts = []
    for half in range(2):
        sims = list(range(half * args.sims, (half + 1) * args.sims))
        h, _, _, _ = sweep.run_batched(held, record=True, tune=False, log=log, sims=sims)
        parts.append(h)
    hh = np.concatenate(parts, axis=1)
    times = list(range(0, cfg.iters - surrogate.HORIZON + 1, 50))
    xe, ye, h0 = surrogate.eval_windows(held, hh, times)
    pred = model.predict(xe)
    lin = surrogate.Linear(x, y)
    pred_lin = lin.predict(xe)
    j_mlp, j_pers, j_lin = (surrogate.judge(p, ye, h0) for p in (pred, h0, pred_lin))
    log(f"[bench] held-out relative L2 error: surrogate {j_mlp}, persistence {j_pers}, linear {j_lin}")
    rg_true = surrogate.r_gyr_from_hist(ye)
    rg_err = np.abs(surrogate.r_gyr_from_hist(pred) - rg_true) / np.maximum(rg_true, 1e-30)
    rg_err_p = np.abs(surrogate.r_gyr_from_hist(h0) - rg_true) / np.maximum(rg_true, 1e-30)
    # screening: 50 iterations for all held-out sets, batched and per simulation, vs one inference
    t_b = 0.0
    for half in range(2):
        sims = list(range(half * args.sims, (half + 1) * args.sims))
        _, tb, _, _ = sweep.run_batched(held, record=False, tune=False, sims=sims, iters=surrogate.HORIZON)
        t_b += tb
    n_ps = min(64, held.n_sims)
    t_ps = float(sweep.run_per_sim(held, list(range(n_ps)), iters=surrogate.HORIZON).sum()) * held.n_sims / n_ps
    # screening cost of the surrogate: one network call on standardised inputs already on the GPU
    x_screen = torch.as_tensor(((xe[:held.n_sims] - model.xm) / model.xs).astype(np.float32), device="cuda")
    x_big = torch.as_tensor(((np.resize(xe, (4096, xe.shape[1])) - model.xm) / model.xs).astype(np.float32),
                            device="cuda")
    net = model.model
    for xx in (x_screen, x_big):
        net.infer(xx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        net.infer(x_screen)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        net.infer(x_big)
    torch.cuda.synchronize()
    t_inf_big = (time.perf_counter() - t0) / reps
    flops = 2.0 * sum(surrogate.DIMS[i] * surrogate.DIMS[i + 1] for i in range(len(surrogate.DIMS) - 1)) * 4096
    screen = screening(args, held, hh, model, t_b, t_ps)
    out = {
        "metric": "surrogate screening speedup over the batched simulation at the stated error",
        "value": t_b / t_inf, "unit": "x", "n_gpus": 1, "steps": args.train_steps, "warmup": 0,
        "ms_per_step": t_train / args.train_steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 (fp32 accumulate)", "data": "synthetic",
        "config": {"workload": f"MLP 35-256-256-256-32 on 20000 windows of a {cfg.n_sims}-simulation sweep "
                               f"(seed 4); judged on {held.n_sims} held-out sets (seed 5) at t = {times}, "
                               f"horizon {surrogate.HORIZON} iterations"},
        "error_rel_l2": {"surrogate": j_mlp, "persistence": j_pers, "linear": j_lin,
                         "r_gyr_rel_median": float(np.median(rg_err)),
                         "r_gyr_rel_median_persistence": float(np.median(rg_err_p))},
        "gain_vs_persistence": {"mean": j_pers["mean"] / j_mlp["mean"],
                                "median_changing": j_pers["median_changing"] / j_mlp["median_changing"],
                                "median": j_pers["median"] / j_mlp["median"]},
        "gain_vs_linear": {"mean": j_lin["mean"] / j_mlp["mean"], "median": j_lin["median"] / j_mlp["median"]},
        "screen_s": {"batched_sim": t_b, "per_simulation_sim": t_ps, "surrogate_infer": t_inf},
        "speedup_vs_per_simulation": t_ps / t_inf,
        "inference_4096": {"ms": t_inf_big * 1e3, "tflops": flops / t_inf_big / 1e12},
        "training_s": t_train,
        "screen_with_fallback": screen,
    }
    print(json.dumps(out), flush=True)


SCREEN_TARGET = 0.02  # mean relative L2 error of the screened histograms


def screening(args, held, hh, model, t_all, t_ps_all):
    """Screening the held-out sweep 50 iterations ahead from its initial
    state, with the plain simulation as fallback: the surrogate predicts every
    set, the sets whose predicted change exceeds a threshold are simulated
    instead (batched), the rest keep the prediction.  The threshold is the
    largest that keeps the mean error within SCREEN_TARGET on the first half
    of the sets; it is applied to the second half, where the end-to-end time
    (inputs to screened histograms) and the error against the full simulation
    of every set are reported.  t_all, t_ps_all: batched and per-simulation
    simulation of all sets."""
    import numpy as np
    import torch
    from paper_2503_10796_amd import sweep, surrogate
    H = surrogate.HORIZON
    n = held.n_sims
    xe = np.concatenate([held.params_unit, np.log1p(hh[0])], axis=1).astype(np.float32)
    truth = hh[H].astype(np.float64)
    pred = model.predict(xe)
    change = surrogate.predicted_change(xe, pred)
    err = surrogate.rel_err(pred, truth)
    pick, judge_sets = np.arange(n // 2), np.arange(n // 2, n)
    tau, frac_pick = surrogate.pick_threshold(change[pick], err[pick], SCREEN_TARGET)
    # end to end on the second half: inference from host inputs, flags, fallback simulation
    xs = xe[judge_sets]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p2 = model.predict(xs)
    flag = surrogate.predicted_change(xs, p2) > tau
    t_pred = time.perf_counter() - t0
    flagged = [int(judge_sets[k]) for k in np.nonzero(flag)[0]]
    t_fb = 0.0
    final = p2.copy()
    if flagged:
        hf, t_fb, _, _ = sweep.run_batched(held, record=True, tune=False, sims=flagged, iters=H)
        assert np.array_equal(hf[H], hh[H][flagged]), "fallback histograms differ from the full simulation"
        final[np.nonzero(flag)[0]] = hf[H]
    e_final = surrogate.rel_err(final, truth[judge_sets])
    e_pred = surrogate.rel_err(p2, truth[judge_sets])
    t_screen = t_pred + t_fb
    t_all_half = t_all * len(judge_sets) / n
    t_ps_half = t_ps_all * len(judge_sets) / n
    # other error targets: threshold from the first half, fallback simulated on the second
    tradeoff = []
    for target in (0.05, 0.10):
        tau2, _ = surrogate.pick_threshold(change[pick], err[pick], target)
        fl2 = [int(judge_sets[k]) for k in np.nonzero(surrogate.predicted_change(xs, p2) > tau2)[0]]
        fin2 = p2.copy()
        t2 = 0.0
        if fl2:
            hf2, t2, _, _ = sweep.run_batched(held, record=True, tune=False, sims=fl2, iters=H)
            fin2[[judge_sets.tolist().index(f) for f in fl2]] = hf2[H]
        e2 = surrogate.rel_err(fin2, truth[judge_sets])
        tradeoff.append({"target_mean_rel_l2": target, "simulated": len(fl2), "mean_error": float(e2.mean()),
                         "seconds": t_pred + t2, "speedup_vs_simulating_all": t_all_half / (t_pred + t2)})
    log(f"[bench] screen: threshold {tau:.4f}, {len(flagged)} of {len(judge_sets)} sets simulated, "
        f"mean error {e_final.mean():.4f} (surrogate alone {e_pred.mean():.4f}), {t_screen:.3f} s vs "
        f"{t_all_half:.3f} s simulating all")
    return {"target_mean_rel_l2": SCREEN_TARGET, "threshold_predicted_change": tau,
            "fallback_fraction_pick_half": frac_pick, "sets": len(judge_sets), "simulated": len(flagged),
            "final_error_rel_l2": {"mean": float(e_final.mean()), "median": float(np.median(e_final)),
                                   "max": float(e_final.max())},
            "surrogate_alone_error_rel_l2": {"mean": float(e_pred.mean()), "median": float(np.median(e_pred)),
                                             "max": float(e_pred.max())},
            "seconds": {"screen": t_screen, "predict_and_flag": t_pred, "fallback_simulation": t_fb,
                        "simulate_all_batched": t_all_half},
            "speedup_vs_simulating_all": t_all_half / t_screen if t_screen > 0 else None,
            "speedup_vs_per_simulation": t_ps_half / t_screen if t_screen > 0 else None,
            "other_targets": tradeoff}


# Sweep work groups per workload, from a scan of 1,024 to 4,096 on one MI355X
# (1,024 is one resident block per LDS slot of the 256 CUs).
SWEEP_GRID = {"uniform": 1024, "relaxed": 2048}


def mechanics_population(kind, agents, resort_every=10, sweep_grid=None, record=False):
    """The mechanics workload at scale, in the launch configuration that is
    timed: (population, agents, description, sweep work groups).  The
    full-size parity tests build their population through this function as
    well, with record=True (the same kernels also write each agent's force
    and counts)."""
    from paper_2503_10796_amd import abm, inputs

    if kind == "uniform":
        pos, diam = inputs.at_density(agents, seed=1)
        side = inputs.cube_side(agents)
        workload = (f"plain mechanics: {agents} agents uniform in a {side:.1f} um cube (1 per 1000 um^3), "
                    f"diameters U[10,15) um, box 15 um, Morton re-sort every {resort_every} iterations")
    else:
        n_side = round(agents ** (1.0 / 3.0))
        pos, diam = inputs.relaxed_lattice(n_side, seed=2)
        side = n_side * 15.5
        workload = (f"pre-relaxed mechanics: {n_side}^3 agents on a jittered 15.5 um lattice with 5% moved next to a "
                    f"neighbour, diameters U[10,15) um, box 15 um, static skip on, Morton re-sort every "
                    f"{resort_every} iterations")
    n = pos.shape[0]
    dims = side / 15.0 + 4.0
    box_cap = int(1.1 * dims ** 3) + 4096
    p = abm.params(box_len=15.0, resort_every=resort_every, detect_static=(kind == "relaxed"), record=record)
    pop = abm.Population(p, pos, diam, capacity=n, box_capacity=box_cap)
    del pos, diam
    if sweep_grid is None:
        sweep_grid = SWEEP_GRID[kind]
    pop.set_sweep_grid(sweep_grid)
    return pop, n, workload, sweep_grid


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--agents", type=int, default=100_000_000)
    ap.add_argument("--workload", choices=["uniform", "relaxed", "sweep", "surrogate", "spheroid", "apoptosis", "sir",
                                           "soma"],
                    default="uniform",
                    help="uniform / relaxed: mechanics at scale (the headline line); sweep: batched parameter "
                         "sweep vs the per-simulation path; surrogate: screening speedup and error; spheroid: "
                         "one tumour spheroid grown to about 5e6 agents; apoptosis: the uniform population with "
                         "the Brownian step and apoptosis of Algorithm 2; sir: Table 4.5's large-scale measles "
                         "epidemic (use --steps 1000); soma: Table 5.1's cell clustering with diffusion")
    ap.add_argument("--soma-resolution", type=int, default=None,
                    help="soma: grid points per axis (default 300, Table 5.1)")
    ap.add_argument("--soma-cpu-iters", type=int, default=1000)
    ap.add_argument("--sir-scale", type=int, default=5000,
                    help="sir: persons as a multiple of Table 4.3's measles model (5000: 1.01e7 persons)")
    ap.add_argument("--sir-boundary", choices=["toroidal", "closed"], default="toroidal")
    ap.add_argument("--sir-cpu-scale", type=int, default=10)
    ap.add_argument("--sir-cpu-iters", type=int, default=1000)
    ap.add_argument("--spheroid-scale", type=float, default=8.0,
                    help="spheroid: factor on the growth rates (8.0 reaches about 5e6 agents at 600 iterations)")
    ap.add_argument("--spheroid-iters", type=int, default=600, help="spheroid: iterations")
    ap.add_argument("--spheroid-cpu-iters", type=int, default=350)
    ap.add_argument("--sweep-cpu-sims", type=int, default=8)
    ap.add_argument("--sweep-cpu-iters", type=int, default=100)
    ap.add_argument("--sims", type=int, default=256, help="sweep: simulations")
    ap.add_argument("--sweep-iters", type=int, default=300, help="sweep: iterations per simulation")
    ap.add_argument("--batched-only", action="store_true",
                    help="sweep: time the batched path only (for kernel traces), no per-simulation comparison")
    ap.add_argument("--train-steps", type=int, default=3000, help="surrogate: Adam steps")
    ap.add_argument("--early-windows", type=float, default=0.0,
                    help="surrogate: share of training windows drawn with density 1/sqrt(t) (near the start)")
    ap.add_argument("--resort-every", type=int, default=10)
    ap.add_argument("--sweep-grid", type=int, default=None,
                    help="sweep work groups (default: 1024 for uniform, 2048 for relaxed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--static-trace", type=int, default=20,
                    help="relaxed: iterations after the timed region whose static share is reported one by one")
    ap.add_argument("--cpu-sample-agents", type=int, default=4_000_000)
    ap.add_argument("--cpu-sample-iters", type=int, default=8)
    ap.add_argument("--cpu-single-agents", type=int, default=1_000_000)
    ap.add_argument("--cpu-single-iters", type=int, default=4)
    ap.add_argument("--oracle-sample", nargs=3, metavar=("WORKLOAD", "AGENTS", "ITERS"),
                    help="only time the oracle on the host (used for the single-thread cpu_baseline sample)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 2 GiB (reference kernel for the HBM byte counters)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write the HBM bytes per force-sweep launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counter "
                         "files (this workload, then the copy calibration) into " + os.path.relpath(PMC_FILE, ROOT))
    args = ap.parse_args()
    if args.oracle_sample:
        w, na, it = args.oracle_sample
        print(json.dumps(oracle_sample(w, int(na), int(it))), flush=True)
        return
    if args.pmc_summary:
        pmc_summary(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration(torch, args.steps)
        return
    sys.path.insert(0, ROOT)
    if args.workload == "sweep":
        bench_sweep(args)
        return
    if args.workload == "surrogate":
        bench_surrogate(args)
        return
    if args.workload == "spheroid":
        bench_spheroid(args)
        return
    if args.workload == "apoptosis":
        bench_apoptosis(args)
        return
    if args.workload == "sir":
        bench_sir(args)
        return
    if args.workload == "soma":
        bench_soma(args)
        return
    from paper_2503_10796_amd import abm

    abm.lib()
    t_gen = time.perf_counter()
    pop, n, workload, sweep_grid = mechanics_population(args.workload, args.agents, args.resort_every,
                                                        args.sweep_grid)
    log(f"[bench] generated and uploaded {n} agents in {time.perf_counter() - t_gen:.1f} s")
    pop.set_timing(True)  # graphs are captured during the warmup
    torch.cuda.synchronize()
    log(f"[bench] population created; workspace {pop.workspace.numel() / 2**30:.1f} GiB")
    pop.step(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} iterations done")
    pop.sweep_time()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pop.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sweep_ms, n_sweeps = pop.sweep_time()
    elapsed = t1 - t0
    log(f"[bench] timed {args.steps} iterations in {elapsed:.3f} s")
    lo, L, gdims = pop.grid()
    nboxes = int(np.prod(gdims))
    static_frac = float(pop.query(abm.STATIC).mean()) if args.workload == "relaxed" else 0.0
    static_trace = None
    if args.workload == "relaxed":
        # static share per iteration over the next iterations (untimed, one at a time)
        static_trace = []
        for _ in range(args.static_trace):
            pop.step(1)
            static_trace.append(round(float(pop.query(abm.STATIC).mean()), 6))
        log(f"[bench] static fraction over {args.static_trace} further iterations: {static_trace}")
    sweep_avg_s = sweep_ms / max(n_sweeps, 1) / 1e3
    alg_bytes = n * SWEEP_BYTES_PER_AGENT + nboxes * SWEEP_BYTES_PER_BOX
    achieved = alg_bytes / sweep_avg_s / 1e9
    traffic = measured_traffic(n, args.workload)
    value = n * args.steps / elapsed
    out = {
        "metric": "agent updates/s per iteration + % HBM peak; batched/surrogate vs plain at error",
        "value": value,
        "unit": "agent updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": workload, "agents": n, "box_len_um": 15.0, "grid_boxes": nboxes,
                   "static_fraction_end": static_frac, "sweep_workgroups": sweep_grid},
        "static_fraction_per_iteration": static_trace,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_sweep", "kernel_ms": sweep_avg_s * 1e3,
                     "algorithmic_bytes_per_launch": alg_bytes},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
