#!/usr/bin/env python3
"""Benchmark of one mechanics iteration at scale on one MI355X.

Workload (default): plain mechanics, 1e8 agents uniform in a cube at 1 agent
per 1000 um^3, diameters U[10, 15) um, box length 15 um, dt 0.01, k = 2,
gamma = 1, adherence 1.8, mass 0.1, cap 3 um, Morton re-sort every 10
iterations; FP32 forces, FP64 positions.  ``--workload relaxed`` runs the
pre-relaxed lattice (most agents static, static skip on).

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


def cpu_baseline(args):
    """The FP64 oracle as it stands on a bounded sample of the same workload."""
    sys.path.insert(0, ROOT)
    from oracle import sim as osim
    from paper_2503_10796_amd import inputs
    n = args.cpu_sample_agents
    if args.workload == "uniform":
        pos, diam = inputs.at_density(n, seed=1)
        detect = False
    else:
        side = round(n ** (1.0 / 3.0))
        pos, diam = inputs.relaxed_lattice(side, seed=2)
        detect = True
    n = pos.shape[0]
    o = osim.OracleSim(pos, diam, osim.make_params(box_len=15.0, detect_static=detect))
    o.step(1)  # first iteration untimed (initialisation excluded)
    t0 = time.perf_counter()
    o.step(args.cpu_sample_iters)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n * args.cpu_sample_iters / dt, "unit": "agent updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} agents of the same workload (same density and diameters), {args.cpu_sample_iters} "
                      f"iterations after one untimed iteration, FP64, OpenMP over agents, {dt:.1f} s"}


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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--agents", type=int, default=100_000_000)
    ap.add_argument("--workload", choices=["uniform", "relaxed"], default="uniform")
    ap.add_argument("--resort-every", type=int, default=10)
    ap.add_argument("--sweep-grid", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-agents", type=int, default=1_000_000)
    ap.add_argument("--cpu-sample-iters", type=int, default=5)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 2 GiB (reference kernel for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration(torch, args.steps)
        return
    sys.path.insert(0, ROOT)
    from paper_2503_10796_amd import abm, inputs

    abm.lib()
    t_gen = time.perf_counter()
    if args.workload == "uniform":
        pos, diam = inputs.at_density(args.agents, seed=1)
        side = inputs.cube_side(args.agents)
        workload = (f"plain mechanics: {args.agents} agents uniform in a {side:.1f} um cube (1 per 1000 um^3), "
                    f"diameters U[10,15) um, box 15 um, Morton re-sort every {args.resort_every} iterations")
    else:
        n_side = round(args.agents ** (1.0 / 3.0))
        pos, diam = inputs.relaxed_lattice(n_side, seed=2)
        side = n_side * 15.5
        workload = (f"pre-relaxed mechanics: {n_side}^3 agents on a jittered 15.5 um lattice with 5% moved next to a "
                    f"neighbour, diameters U[10,15) um, box 15 um, static skip on, Morton re-sort every "
                    f"{args.resort_every} iterations")
    n = pos.shape[0]
    log(f"[bench] generated {n} agents in {time.perf_counter() - t_gen:.1f} s")
    dims = side / 15.0 + 4.0
    box_cap = int(1.1 * dims ** 3) + 4096
    p = abm.params(box_len=15.0, resort_every=args.resort_every, detect_static=(args.workload == "relaxed"))
    pop = abm.Population(p, pos, diam, capacity=n, box_capacity=box_cap)
    del pos, diam
    pop.set_sweep_grid(args.sweep_grid)
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
                   "static_fraction_end": static_frac, "sweep_workgroups": args.sweep_grid},
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
