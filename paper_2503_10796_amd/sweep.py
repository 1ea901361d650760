"""Batched parameter sweeps of tumour-spheroid growth.

Hundreds of independent simulations (uneven agent counts) advance together
as one batch: one captured graph launch per iteration, launch schedule picked
by the library's autotuner.  The per-simulation path (one Population per
simulation, run one after another) is the baseline the batch is measured
against.  Radial density histograms recorded every iteration feed the
surrogate's training windows.
"""
import math
import time

import numpy as np

from . import abm, inputs

HIST_RMAX = 300.0  # um: radius covered by the 32 histogram shells
ITERS = 300


class SweepConfig:
    """Latin-hypercube sweep: per simulation the initial count n0 (log-uniform),
    growth-rate scale, division diameter and adherence; cells seeded in a ball
    (diameter 8 um, lognormal growth rates of mean 1 um^3/step times the scale)."""

    def __init__(self, n_sims=256, seed=4, iters=ITERS, n_lo=1.0e3, n_hi=5.0e4):
        self.n_sims, self.seed, self.iters = n_sims, seed, iters
        self.n0, self.gscale, self.d_div, self.adherence = inputs.sweep_params(n_sims, seed, n_lo, n_hi)
        self.params_unit = np.stack([(self.gscale - 0.5) / 1.0, (self.d_div - 6.0) / 12.0,
                                     (self.adherence - 0.9) / 1.8], axis=1)

    def state(self, s):
        return inputs.spheroid(int(self.n0[s]), seed=self.seed * 100003 + s, growth_scale=float(self.gscale[s]))

    def params(self, s, resort_every=10, record=False):
        return abm.params(box_len=0.0, div_vol=inputs.division_volume(float(self.d_div[s])),
                          adherence=float(self.adherence[s]), detect_static=True, resort_every=resort_every,
                          seed=self.seed, sim_id=s, record=record)

    def counts(self, s, vol, growth):
        """Agent count of simulation s at every iteration 0..iters.  Growth and
        division of a cell do not depend on positions (grow below the division
        volume, else split into two halves with the same rate), so each lineage
        is followed as (volume, multiplicity) with the same FP64 operations."""
        vdiv = inputs.division_volume(float(self.d_div[s]))
        V = np.array(vol, dtype=np.float64)
        m = np.ones_like(V)
        out = [float(m.sum())]
        for _ in range(self.iters):
            div = V >= vdiv
            V = np.where(div, 0.5 * V, V + growth)
            m = np.where(div, 2.0 * m, m)
            out.append(float(m.sum()))
        return np.array(out)

    def capacity(self, s, vol, growth):
        return int(1.1 * self.counts(s, vol, growth)[-1]) + 1024


def build_batch(cfg, sims=None, resort_every=10, record=False):
    """One Batch holding the given simulations (all by default); record=True
    makes the kernels also write each agent's force and counts (ABM_RECORD)."""
    sims = list(range(cfg.n_sims)) if sims is None else list(sims)
    states = [cfg.state(s) for s in sims]
    caps = [cfg.capacity(s, st[2], st[3]) for s, st in zip(sims, states)]
    bcaps = [3 * c + 65536 for c in caps]
    b = abm.Batch([cfg.params(s, resort_every, record) for s in sims], [st[0].shape[0] for st in states],
                  np.concatenate([st[0] for st in states]), np.concatenate([st[1] for st in states]),
                  vol=np.concatenate([st[2] for st in states]), growth=np.concatenate([st[3] for st in states]),
                  capacity=caps, box_capacity=bcaps)
    return b, states, caps


def run_batched(cfg, record=True, tune=True, log=None, sims=None, iters=None):
    """Runs the sweep (or the listed simulations) batched for `iters`
    iterations (cfg.iters by default); returns (histograms [iters+1, n, 32] or
    None, seconds for the iterations, agents per simulation at the end,
    launch schedule).  With tune=True the autotuner picks the schedule,
    including the Morton re-sort period; else the re-sort runs every 10
    iterations."""
    import torch
    iters = cfg.iters if iters is None else iters
    sims = list(range(cfg.n_sims)) if sims is None else list(sims)
    b, _, _ = build_batch(cfg, sims, resort_every=-1 if tune else 10)
    if tune:
        b.tune(3)
    grid = b.schedule()
    torch.cuda.synchronize()
    hist = torch.zeros((iters + 1, len(sims), 32), dtype=torch.float32, device="cuda") if record else None
    if record:
        b.hist_device(hist[0], HIST_RMAX)
    for it in range(iters):
        if it == 1:  # the first iteration (graph capture) is excluded from the timing
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        b.step(1)
        if record:
            b.hist_device(hist[it + 1], HIST_RMAX)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) * iters / (iters - 1)
    n_end = b.num_agents()
    if log:
        log(f"[sweep] {len(sims)} simulations x {iters} its batched in {dt:.3f} s, "
            f"{int(n_end.sum())} agents at the end, schedule {grid}")
    out = hist.cpu().numpy() if record else None
    b.close()
    return out, dt, n_end, grid


def run_per_sim(cfg, sims, log=None, iters=None):
    """The per-simulation path: each simulation as its own Population, one
    after another, for `iters` iterations (cfg.iters by default).  Returns
    seconds per simulation."""
    import torch
    iters = cfg.iters if iters is None else iters
    secs = []
    for s in sims:
        pos, diam, vol, growth = cfg.state(s)
        cap = cfg.capacity(s, vol, growth)
        p = abm.Population(cfg.params(s), pos, diam, vol=vol, growth=growth, capacity=cap, box_capacity=3 * cap + 65536)
        p.step(1)  # graph capture and first launch excluded, as for the batch
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.step(iters - 1)
        torch.cuda.synchronize()
        secs.append((time.perf_counter() - t0) * iters / (iters - 1))
        p.close()
        if log:
            log(f"[sweep] per-simulation path: sim {s} (n0 {cfg.n0[s]}) {secs[-1]:.3f} s")
    return np.array(secs)


def stratified_sample(cfg, k):
    """k simulations spread over the range of initial counts (for timing the
    per-simulation path on a sample)."""
    order = np.argsort(cfg.n0)
    idx = np.linspace(0, cfg.n_sims - 1, k).round().astype(int)
    return sorted(set(int(order[i]) for i in idx))
