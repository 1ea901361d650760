"""Pins of the SIR epidemiology oracle (Algorithms 3-5, Sec 4.4.11, Table 4.3)
against what the paper and the mathematics fix: the SIR differential
equations the thesis compares its model with (Fig 4.17), binomial closed
forms of the recovery and infection draws, an independent enumeration of the
torus images for the neighbourhood, and invariants of the movement and the
boundaries."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import sir
from paper_2503_10796_amd import inputs


def _ode(cfg, steps):
    """The SIR equations (dS/dt = -beta S I / N, dI/dt = beta S I / N - gamma I,
    dR/dt = gamma I) with Table 4.3's beta and gamma, one time unit per step."""
    n = cfg["n_susceptible"] + cfg["n_infected"]
    b, g = cfg["beta"], cfg["gamma"]

    def f(_, y):
        return [-b * y[0] * y[1] / n, b * y[0] * y[1] / n - g * y[1], g * y[1]]

    y0 = [cfg["n_susceptible"], cfg["n_infected"], 0.0]
    return solve_ivp(f, (0, steps), y0, t_eval=np.arange(steps + 1), rtol=1e-10, atol=1e-8).y.T / n


def _run(cfg, seed, steps=None, boundary=sir.TOROIDAL):
    steps = cfg["steps"] if steps is None else steps
    pos, st = inputs.sir_population(cfg["n_susceptible"], cfg["n_infected"], cfg["space"], seed=seed)
    p = sir.make_params(cfg["space"], cfg["radius"], cfg["infection_prob"], cfg["recovery_prob"], cfg["speed"],
                        boundary=boundary, seed=seed)
    o = sir.OracleSIR(pos, st, p)
    h = o.step(steps)
    n = pos.shape[0]
    return np.vstack([[cfg["n_susceptible"], cfg["n_infected"], 0], h]) / n, o


def test_measles_follows_the_sir_equations():
    """Table 4.3 measles (2,000 + 20 persons, 1,000 steps), mean of four
    seeds: the infected curve follows the SIR equations with beta = 0.06719
    and gamma = 0.00521 (R0 = 12.9): peak share (0.725) within 0.03, peak
    step (117) within 10, the largest gap of the infected share below 0.1,
    and nearly everyone recovered at the end (Fig 4.17A)."""
    cfg = inputs.SIR_MEASLES
    y = _ode(cfg, cfg["steps"])
    runs = [_run(cfg, seed)[0] for seed in range(4)]
    m = np.mean(runs, axis=0)
    assert abs(m[:, 1].max() - y[:, 1].max()) <= 0.03, (m[:, 1].max(), y[:, 1].max())
    assert abs(int(m[:, 1].argmax()) - int(y[:, 1].argmax())) <= 10
    assert np.abs(m[:, 1] - y[:, 1]).max() <= 0.1
    assert m[-1, 2] >= 0.98 and y[-1, 2] >= 0.98
    # the closed-form peak of the SIR equations, 1 - (1 + ln R0) / R0 (S0 ~ N)
    r0 = cfg["beta"] / cfg["gamma"]
    s0 = cfg["n_susceptible"] / (cfg["n_susceptible"] + cfg["n_infected"])
    peak = 1.0 - (1.0 + math.log(r0 * s0)) / r0
    assert abs(y[:, 1].max() - peak) <= 1e-3


def test_influenza_follows_the_sir_equations():
    """Table 4.3 seasonal influenza (20,000 + 200 persons, 2,500 steps,
    R0 = 1.3): peak infected share (0.0366 at step 770) within 0.005 and 100
    steps, final recovered share (0.441 from the equations; the final-size
    relation 1 - x = exp(-R0 x) gives 0.44 too) within 0.04 (Fig 4.17B)."""
    cfg = inputs.SIR_INFLUENZA
    y = _ode(cfg, cfg["steps"])
    m, _ = _run(cfg, 0)
    assert abs(m[:, 1].max() - y[:, 1].max()) <= 0.005
    assert abs(int(m[:, 1].argmax()) - int(y[:, 1].argmax())) <= 100
    assert abs(m[-1, 2] - y[-1, 2]) <= 0.04
    r0 = cfg["beta"] / cfg["gamma"]
    x = 0.5
    for _ in range(200):  # final size of the SIR equations: 1 - x = s0 exp(-R0 x)
        x = 1.0 - 0.990099 * math.exp(-r0 * x)
    assert abs(y[-1, 2] - x) <= 0.01


def test_counts_are_conserved_and_monotone():
    cfg = inputs.SIR_MEASLES
    m, o = _run(cfg, 5, steps=300)
    assert np.allclose(m.sum(axis=1), 1.0)
    assert np.all(np.diff(m[:, 0]) <= 0) and np.all(np.diff(m[:, 2]) >= 0)
    assert np.array_equal(o.counts(), np.rint(m[-1] * o.n).astype(np.int64))


def test_recovery_alone_is_binomial():
    """No infection (probability 0): after t steps each infected person is
    still infected with probability (1 - p)^t, independently (Algorithm 4)."""
    n, p_rec, t = 20000, 0.01, 50
    pos = np.random.default_rng(1).uniform(0, 50.0, size=(n, 3))
    st = np.ones(n, dtype=np.uint8)
    o = sir.OracleSIR(pos, st, sir.make_params(50.0, 2.0, 0.0, p_rec, 1.0, seed=3))
    h = o.step(t)
    q = (1.0 - p_rec) ** t
    mean, sd = n * q, math.sqrt(n * q * (1 - q))
    assert abs(h[-1, 1] - mean) <= 5 * sd, (h[-1, 1], mean, sd)
    assert h[-1, 0] == 0 and h[-1, 1] + h[-1, 2] == n


def test_infection_with_everyone_in_range_is_binomial():
    """An infection radius beyond the largest torus distance (S sqrt(3) / 2)
    puts every infected person in range of everyone: each susceptible person
    is infected with probability p per step, so after t steps
    S_t ~ Binomial(S_0, (1 - p)^t) (Algorithm 3)."""
    n_s, n_i, p_inf, t, space = 20000, 10, 0.05, 20, 20.0
    pos, st = inputs.sir_population(n_s, n_i, space, seed=2)
    o = sir.OracleSIR(pos, st, sir.make_params(space, space, p_inf, 0.0, 1.0, seed=4))
    h = o.step(t)
    q = (1.0 - p_inf) ** t
    mean, sd = n_s * q, math.sqrt(n_s * q * (1 - q))
    assert abs(h[-1, 0] - mean) <= 5 * sd, (h[-1, 0], mean, sd)


def _images_infected(pos, st, space, r, toroidal):
    """Susceptible persons with an infected one strictly within r, by
    enumerating the 27 periodic images explicitly (toroidal) or the plain
    distance (closed)."""
    shifts = [np.zeros(3)]
    if toroidal:
        shifts = [np.array([a, b, c]) * space for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    inf = pos[st == 1]
    out = np.zeros(pos.shape[0], dtype=bool)
    for i in np.nonzero(st == 0)[0]:
        d2 = min(((inf + s - pos[i]) ** 2).sum(axis=1).min() for s in shifts)
        out[i] = d2 < r * r
    return out


@pytest.mark.parametrize("boundary", [sir.TOROIDAL, sir.CLOSED])
def test_neighbourhood_matches_image_enumeration(boundary):
    """With infection probability 1, no recovery and no movement, one step
    infects exactly the susceptible persons that have an infected person
    within the radius: minimum image on the torus, plain distance in a
    closed space.  Checked against an enumeration of the periodic images."""
    rng = np.random.default_rng(7)
    n, space, r = 400, 12.0, 2.5
    pos = rng.uniform(0, space, size=(n, 3))
    st = (rng.random(n) < 0.1).astype(np.uint8)
    expect = _images_infected(pos, st, space, r, boundary == sir.TOROIDAL)
    o = sir.OracleSIR(pos, st, sir.make_params(space, r, 1.0, 0.0, 0.0, boundary=boundary, seed=1))
    o.step(1)
    got = (o.state == 1) & (st == 0)
    assert np.array_equal(got, expect)
    assert 20 < expect.sum() < (st == 0).sum()
    assert np.array_equal(o.pos(), pos)  # speed 0: nobody moves


def test_radius_is_strict_and_closed_space_does_not_wrap():
    space, r = 10.0, 2.0
    # exactly r apart along x: not within the radius
    pos = np.array([[1.0, 5.0, 5.0], [3.0, 5.0, 5.0]])
    o = sir.OracleSIR(pos, np.array([0, 1], np.uint8), sir.make_params(space, r, 1.0, 0.0, 0.0))
    o.step(1)
    assert o.state[0] == 0
    # 1.5 apart across the x faces: in range on the torus only
    pos = np.array([[0.5, 5.0, 5.0], [9.0, 5.0, 5.0]])
    for boundary, expect in ((sir.TOROIDAL, 1), (sir.CLOSED, 0)):
        o = sir.OracleSIR(pos, np.array([0, 1], np.uint8), sir.make_params(space, r, 1.0, 0.0, 0.0,
                                                                           boundary=boundary))
        o.step(1)
        assert o.state[0] == expect, boundary
    assert sir.dist2((0.5, 5, 5), (9.0, 5, 5), space, sir.TOROIDAL) == 2.25
    assert sir.dist2((0.5, 5, 5), (9.0, 5, 5), space, sir.CLOSED) == 72.25


def test_random_step_length_and_moments():
    """Algorithm 5: the step is the normalised cube vector times the speed:
    length = speed (to rounding), components of mean 0 and mean square
    speed^2 / 3 (symmetry of the cube)."""
    speed = 5.78594
    d = np.array([sir.step_vector(9, 0, u, 3, speed) for u in range(20000)])
    assert np.allclose(np.linalg.norm(d, axis=1), speed, rtol=1e-15, atol=0)
    assert np.all(np.abs(d.mean(axis=0)) < 5 * speed / math.sqrt(3 * 20000))
    assert np.allclose((d ** 2).mean(axis=0), speed ** 2 / 3, rtol=0.03)
    # independent streams per uid and iteration
    assert not np.array_equal(sir.step_vector(9, 0, 1, 3, speed), sir.step_vector(9, 0, 1, 4, speed))


def test_boundaries_closed_form():
    s = 100.0
    assert sir.bound(100.5, s, sir.TOROIDAL) == 0.5
    assert sir.bound(-0.25, s, sir.TOROIDAL) == 99.75
    assert sir.bound(42.0, s, sir.TOROIDAL) == 42.0
    assert sir.bound(-1e-300, s, sir.TOROIDAL) == 100.0  # S + tiny rounds to S: the face itself
    assert sir.bound(-0.25, s, sir.CLOSED) == 0.0
    assert sir.bound(100.5, s, sir.CLOSED) == 100.0
    assert sir.bound(42.0, s, sir.CLOSED) == 42.0


@pytest.mark.parametrize("boundary", [sir.TOROIDAL, sir.CLOSED])
def test_movement_stays_in_the_space(boundary):
    cfg = inputs.SIR_MEASLES
    pos, st = inputs.sir_population(500, 5, 20.0, seed=3)
    o = sir.OracleSIR(pos, st, sir.make_params(20.0, 1.0, 0.0, 0.0, cfg["speed"], boundary=boundary, seed=8))
    for it in range(5):
        p0 = o.pos().copy()
        o.step(1)
        p1 = o.pos()
        assert np.all((p1 >= 0) & (p1 <= 20.0))
        d = np.array([sir.step_vector(8, 0, u, it, cfg["speed"]) for u in range(o.n)])
        if boundary == sir.TOROIDAL:
            off = p1 - p0
            off -= 20.0 * np.rint(off / 20.0)
            assert np.allclose(off, d, atol=1e-12)
        else:
            assert np.allclose(p1, np.clip(p0 + d, 0.0, 20.0), atol=1e-12, rtol=0)
