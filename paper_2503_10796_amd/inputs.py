"""Seeded synthetic inputs shared by the HIP path's tests/benchmarks and the oracle.

This module holds no arithmetic of the method: it only draws populations
(positions, diameters, volumes, growth rates) and sweep parameters from
seeded numpy generators.  Every workload is synthetic; the thesis measures
on no public dataset for this path.

Recipes (sizes and distributions of the thesis's tissue benchmarks):
  plain(n, side, seed)      centres uniform in [0, side)^3, diameters U[10, 15)
  at_density(n, seed)       same, side chosen for 1 agent per 1000 um^3
  relaxed_lattice(n, seed)  jittered cubic lattice (spacing 15.5 um, jitter 0.2 um,
                            diameters U[10, 15)) with 5 % of agents moved 8-12 um
                            from a lattice neighbour, so most agents start static
  spheroid(n, seed, ...)    centres uniform in a ball (radius 50 um at 1000 cells,
                            constant density otherwise), diameter 8 um, volume
                            pi d^3 / 6, growth rate lognormal with arithmetic
                            mean 1 and log-sd 0.2 (um^3 per step)
  sweep_params(n, seed)     Latin hypercube over growth scale [0.5, 1.5],
                            division diameter [6, 18] um, adherence [0.9, 2.7],
                            and log-uniform initial counts in [1e3, 5e4]
  sir_population(...)       persons uniform in a cube of side S (metres), the
                            first n_infected infected, the rest susceptible;
                            SIR_MEASLES / SIR_INFLUENZA hold the Table 4.3
                            sizes and parameters, scaled_sir() the same density
                            at k times the persons
  soma_population(cfg)      cells uniform in the cubic space, types alternating
                            0, 1; SOMA_CELL_CLUSTERING holds Table 5.1's cell
                            clustering sizes (2e6 cells, two substances on
                            300^3 points)
"""
import math

import numpy as np

DENSITY = 1.0e-3  # agents per um^3


def plain(n, side=160.0, seed=0, dmin=10.0, dmax=15.0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, side, size=(n, 3))
    diam = rng.uniform(dmin, dmax, size=n)
    return pos, diam


def cube_side(n, density=DENSITY):
    return (n / density) ** (1.0 / 3.0)


def at_density(n, seed=1, density=DENSITY):
    return plain(n, side=cube_side(n, density), seed=seed)


def relaxed_lattice(n_side, seed=2, spacing=15.5, jitter=0.2, frac_moved=0.05):
    """Pre-relaxed population: a jittered lattice where no pair touches, plus a
    random 5 % of agents moved along a lattice line to 8-12 um from a lattice
    neighbour.  Returns pos, diam."""
    rng = np.random.default_rng(seed)
    g = np.arange(n_side, dtype=np.float64) * spacing
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    n = pos.shape[0]
    pos += rng.uniform(-jitter, jitter, size=pos.shape)
    diam = rng.uniform(10.0, 15.0, size=n)
    moved = rng.random(n) < frac_moved
    idx = np.nonzero(moved)[0]
    axis = rng.integers(0, 3, size=idx.size)
    sign = rng.choice([-1.0, 1.0], size=idx.size)
    gap = rng.uniform(8.0, 12.0, size=idx.size)
    # move towards the chosen neighbour so that it sits `gap` away from it
    pos[idx, axis] += sign * (spacing - gap)
    return pos, diam


def ball(n, radius, rng):
    out = np.empty((0, 3))
    while out.shape[0] < n:
        c = rng.uniform(-radius, radius, size=(2 * n, 3))
        c = c[(c * c).sum(axis=1) < radius * radius]
        out = np.concatenate([out, c], axis=0)
    return out[:n]


def spheroid(n=1000, seed=3, diameter=8.0, growth_mean=1.0, growth_sigma=0.2, growth_scale=1.0,
             radius=None):
    rng = np.random.default_rng(seed)
    if radius is None:
        radius = 50.0 * (n / 1000.0) ** (1.0 / 3.0)
    pos = ball(n, radius, rng)
    diam = np.full(n, diameter)
    vol = np.full(n, math.pi * diameter ** 3 / 6.0)
    mu = math.log(growth_mean) - 0.5 * growth_sigma ** 2
    growth = rng.lognormal(mean=mu, sigma=growth_sigma, size=n) * growth_scale
    return pos, diam, vol, growth


def division_volume(d_div):
    return math.pi * d_div ** 3 / 6.0


def sweep_params(n_sims, seed=4, n_lo=1.0e3, n_hi=5.0e4):
    """Latin-hypercube sweep: one stratum per simulation in every dimension."""
    rng = np.random.default_rng(seed)
    n0 = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=n_sims))).astype(np.int64)

    def lhs(lo, hi):
        perm = rng.permutation(n_sims)
        u = (perm + rng.random(n_sims)) / n_sims
        return lo + (hi - lo) * u

    gscale = lhs(0.5, 1.5)
    d_div = lhs(6.0, 18.0)
    adherence = lhs(0.9, 2.7)
    return n0, gscale, d_div, adherence


# Table 4.3: cubic space length (m), persons (susceptible, infected), infection
# radius (m), infection and recovery probabilities, maximum movement per step
# (m), time steps; beta and gamma of the SIR equations it is compared with.
SIR_MEASLES = dict(space=100.0, n_susceptible=2000, n_infected=20, radius=3.24179, infection_prob=0.28510,
                   recovery_prob=0.00521, speed=5.78594, steps=1000, beta=0.06719, gamma=0.00521)
SIR_INFLUENZA = dict(space=215.0, n_susceptible=20000, n_infected=200, radius=3.2123, infection_prob=0.04980,
                     recovery_prob=0.01016, speed=4.2942, steps=2500, beta=0.01321, gamma=0.01016)


def scaled_sir(cfg, k):
    """The same model at k times the persons and the same density."""
    out = dict(cfg)
    out["n_susceptible"] = int(cfg["n_susceptible"] * k)
    out["n_infected"] = int(cfg["n_infected"] * k)
    out["space"] = cfg["space"] * float(k) ** (1.0 / 3.0)
    return out


def sir_population(n_susceptible, n_infected, space, seed=0):
    """Positions uniform in [0, space)^3 (float64, n x 3) and states (uint8:
    0 susceptible, 1 infected); persons 0..n_infected-1 start infected."""
    n = int(n_susceptible) + int(n_infected)
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, space, size=(n, 3))
    state = np.zeros(n, dtype=np.uint8)
    state[: int(n_infected)] = 1
    return pos, state


# Table 5.1, cell clustering: 2e6 cells and 54 million diffusion volumes (two
# substances on 300^3 points), 1,000 iterations.  The thesis gives the
# secretion quantity (1) and the gradient weight (0.75) of the model
# (Sec 4.7.1); the space (1,200 um: 4 um voxels, 1.16 cells per 1000 um^3),
# diffusion coefficient, decay and time step are chosen here
# (stable: 6 nu dt / dx^2 = 0.375).
SOMA_CELL_CLUSTERING = dict(lo=0.0, space=1200.0, resolution=300, n_substances=2, diffusion=1.0, decay=0.01,
                            dt=1.0, secretion=1.0, gradient_weight=0.75, n_cells=2_000_000, steps=1000)


def soma_population(cfg, seed=0):
    """Cell positions uniform in the cubic space (float64, n x 3) and types
    (int32) alternating over the substances."""
    rng = np.random.default_rng(seed)
    n = int(cfg["n_cells"])
    pos = cfg["lo"] + rng.uniform(0.0, cfg["space"], size=(n, 3))
    t = (np.arange(n) % int(cfg["n_substances"])).astype(np.int32)
    return pos, t
