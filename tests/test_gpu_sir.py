"""SIR epidemiology on the GPU (Algorithms 3-5, Sec 4.4.11, Table 4.3)
against the oracle.  Every decision is an integer outcome of FP64 arithmetic
that both sides evaluate in the same IEEE operations, so the comparison is
exact: counts per iteration, every person's state, and every coordinate bit
for bit (persons matched by uid)."""
import time

import numpy as np
import pytest

from oracle import sir as osir
from paper_2503_10796_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10796_amd import abm as _abm
    _abm.lib()
    return _abm


def _params(abm, cfg, seed, boundary=0, **kw):
    base = dict(space=cfg["space"], radius=cfg["radius"], infection_prob=cfg["infection_prob"],
                recovery_prob=cfg["recovery_prob"], speed=cfg["speed"])
    base.update(kw)
    gp = abm.sir_params(base["space"], base["radius"], base["infection_prob"], base["recovery_prob"], base["speed"],
                        boundary=boundary, seed=seed)
    op = osir.make_params(base["space"], base["radius"], base["infection_prob"], base["recovery_prob"],
                          base["speed"], boundary=boundary, seed=seed)
    return gp, op


def _same_state(abm, g, o, what):
    uid = g.query(abm.SIR_UID).astype(np.int64)
    assert np.array_equal(np.sort(uid), np.arange(o.n)), what
    inv = np.empty(o.n, dtype=np.int64)
    inv[uid] = np.arange(o.n)
    st = g.query(abm.SIR_STATE)[inv]
    pos = g.query(abm.SIR_POS)[inv]
    assert np.array_equal(st, o.state), f"{what}: {int((st != o.state).sum())} states differ"
    assert np.array_equal(pos, o.pos()), f"{what}: positions differ (max {np.abs(pos - o.pos()).max():.3e})"


def _run_pair(abm, cfg, seed, iters, every, boundary=0, **kw):
    pos, st = inputs.sir_population(cfg["n_susceptible"], cfg["n_infected"], cfg["space"], seed=seed)
    gp, op = _params(abm, cfg, seed, boundary, **kw)
    g = abm.Sir(gp, pos, st, hist_cap=256)
    o = osir.OracleSIR(pos, st, op)
    _same_state(abm, g, o, "initial")
    done = 0
    while done < iters:
        k = min(every, iters - done)
        hg = g.step(k, counts=True)
        ho = o.step(k)
        assert np.array_equal(hg, ho), f"counts differ in iterations {done}..{done + k}"
        done += k
        _same_state(abm, g, o, f"iteration {done}")
    return g, o


def test_measles_matches_oracle(abm):
    """Table 4.3 measles (2,000 + 20 persons, toroidal space of 100 m),
    1,000 iterations: counts after every iteration equal, states and
    positions bit for bit every 100 iterations (the run of Fig 4.17A)."""
    cfg = inputs.SIR_MEASLES
    t0 = time.perf_counter()
    g, o = _run_pair(abm, cfg, seed=0, iters=cfg["steps"], every=100)
    it, c = g.counts()
    assert it == cfg["steps"] and np.array_equal(c, o.counts())
    assert c[2] > 0.95 * o.n  # the epidemic ran its course
    print(f"measles: 1000 iterations equal, final {c.tolist()}, {time.perf_counter() - t0:.1f} s", flush=True)


def test_closed_space_matches_oracle(abm):
    """The measles model in a closed space (walls clamp the persons), 300
    iterations."""
    cfg = inputs.SIR_MEASLES
    _run_pair(abm, cfg, seed=3, iters=300, every=50, boundary=1)


def test_influenza_matches_oracle(abm):
    """Table 4.3 seasonal influenza (20,000 + 200 persons, 215 m), the first
    600 iterations (rising to the peak of Fig 4.17B)."""
    cfg = inputs.SIR_INFLUENZA
    _run_pair(abm, cfg, seed=1, iters=600, every=150)


@pytest.mark.parametrize("case", ["one_box", "two_boxes", "faces", "coincident", "certain_infection", "static"])
def test_edge_cases_match_oracle(abm, case):
    """Degenerate grids and inputs: a space smaller than six radii (one box
    per axis: boxes are three radii long), two boxes per axis on the torus (both neighbours are the same
    box), persons exactly on the faces of the space, persons at identical
    positions, infection probability 1 without recovery, no movement."""
    rng = np.random.default_rng(11)
    cfg = dict(inputs.SIR_MEASLES)
    n = 600
    if case == "one_box":
        space, kw = 10.0, {}
    elif case == "two_boxes":
        space, kw = 22.0, {}
    elif case == "certain_infection":
        space, kw = 40.0, dict(infection_prob=1.0, recovery_prob=0.0)
    elif case == "static":
        space, kw = 40.0, dict(speed=0.0, infection_prob=1.0)
    else:
        space, kw = 40.0, {}
    pos = rng.uniform(0, space, size=(n, 3))
    if case == "faces":
        pos[:100] = rng.choice([0.0, space], size=(100, 3))
        pos[100:200, 0] = space
    if case == "coincident":
        pos[300:400] = pos[0:100]
    st = (rng.random(n) < 0.05).astype(np.uint8)
    gp, op = _params(abm, cfg, 5, 0, space=space, speed=kw.pop("speed", 3.0), **kw)
    for boundary in (0, 1):
        gp.boundary = op.boundary = boundary
        g = abm.Sir(gp, pos, st, hist_cap=64)
        if case == "one_box":
            assert g.grid()[0] == 1
        if case == "two_boxes":
            assert g.grid()[0] == 2
        o = osir.OracleSIR(pos, st, op)
        for k in range(3):
            assert np.array_equal(g.step(10, counts=True), o.step(10)), (case, boundary, k)
            _same_state(abm, g, o, f"{case}, boundary {boundary}, iteration {10 * (k + 1)}")


def test_empty_population(abm):
    gp, _ = _params(abm, inputs.SIR_MEASLES, 0)
    g = abm.Sir(gp, np.zeros((0, 3)), np.zeros(0, np.uint8), hist_cap=8)
    assert np.array_equal(g.step(20, counts=True), np.zeros((20, 3), np.int64))
    it, c = g.counts()
    assert it == 20 and np.array_equal(c, np.zeros(3))
    assert g.query(abm.SIR_POS).shape == (0, 3)


def test_invalid_inputs_are_refused(abm):
    cfg = inputs.SIR_MEASLES
    pos, st = inputs.sir_population(10, 1, cfg["space"], seed=0)
    gp, _ = _params(abm, cfg, 0)
    bad = pos.copy()
    bad[0, 0] = cfg["space"] * 1.5
    with pytest.raises(abm.AbmError):
        abm.Sir(gp, bad, st)
    bad[0, 0] = np.nan
    with pytest.raises(abm.AbmError):
        abm.Sir(gp, bad, st)
    with pytest.raises(abm.AbmError):
        abm.Sir(gp, pos, np.full(11, 3, np.uint8))
    with pytest.raises(abm.AbmError):  # a toroidal step must be shorter than the space
        abm.Sir(abm.sir_params(10.0, 1.0, 0.5, 0.1, 10.0), np.full((2, 3), 1.0), np.zeros(2, np.uint8))


def test_stepping_granularity_and_timing_do_not_change_results(abm):
    """One call of 120 iterations, 120 calls of one, and the timed path (the
    person kernel between events) give the same persons bit for bit."""
    cfg = inputs.SIR_MEASLES
    pos, st = inputs.sir_population(cfg["n_susceptible"], cfg["n_infected"], cfg["space"], seed=8)
    gp, _ = _params(abm, cfg, 8)
    a = abm.Sir(gp, pos, st)
    a.step(120)
    b = abm.Sir(gp, pos, st)
    for _ in range(120):
        b.step(1)
    c = abm.Sir(gp, pos, st)
    c.set_timing(True)
    hc = c.step(120, counts=True)
    ms, k = c.kernel_time()
    assert k == 120 and ms > 0.0
    for h in (b, c):
        for f in (abm.SIR_STATE, abm.SIR_POS):
            ua, uh = a.query(abm.SIR_UID), h.query(abm.SIR_UID)
            assert np.array_equal(a.query(f)[np.argsort(ua)], h.query(f)[np.argsort(uh)])
    assert np.array_equal(hc[-1], a.counts()[1])


@pytest.mark.timeout(600)
def test_large_scale_sampled_persons_match_oracle(abm):
    """Table 4.5's large-scale measles population (5,000 times Table 4.3:
    1.01e7 persons in a 1,710 m torus) after 80 iterations: one GPU iteration against the oracle's iteration on the
    persons of four cubes of half side 25 m grown by the infection radius
    plus a margin (a corner, so that the cube wraps around the torus, and
    three random ones): every inner person's state and position bit for bit.
    Iteration 80 is in the steep rise of the epidemic."""
    cfg = inputs.scaled_sir(inputs.SIR_MEASLES, 5000)
    t0 = time.perf_counter()
    pos, st = inputs.sir_population(cfg["n_susceptible"], cfg["n_infected"], cfg["space"], seed=12)
    gp, op = _params(abm, cfg, 12, space=cfg["space"])
    g = abm.Sir(gp, pos, st)
    del pos, st
    g.step(80)
    S = cfg["space"]
    p0, s0, u0 = g.query(abm.SIR_POS), g.query(abm.SIR_STATE), g.query(abm.SIR_UID).astype(np.int64)
    counts = np.bincount(s0, minlength=3)
    assert counts[1] > 0.01 * u0.size and counts[0] > 0.05 * u0.size, counts
    g.step(1)
    p1, s1, u1 = g.query(abm.SIR_POS), g.query(abm.SIR_STATE), g.query(abm.SIR_UID).astype(np.int64)
    inv = np.empty(u1.size, dtype=np.int64)
    inv[u1] = np.arange(u1.size)
    rng = np.random.default_rng(5)
    half, grow = 25.0, cfg["radius"] + 1.0
    checked = infected_now = 0
    for c in [np.zeros(3)] + [rng.uniform(0, S, 3) for _ in range(3)]:
        off = p0 - c
        off -= S * np.rint(off / S)  # minimum image
        near = np.all(np.abs(off) < half + grow, axis=1)
        sel = np.nonzero(near)[0]
        o = osir.OracleSIR(p0[sel], s0[sel], op, uid=u0[sel].astype(np.uint64), iteration=80)
        o.step(1)
        inner = np.all(np.abs(off[sel]) < half, axis=1)
        gi = inv[u0[sel][inner]]
        assert np.array_equal(s1[gi], o.state[inner])
        assert np.array_equal(p1[gi], o.pos()[inner])
        checked += int(inner.sum())
        infected_now += int(((s0[sel][inner] == 0) & (o.state[inner] != 0)).sum())
    print(f"large scale: {u0.size} persons, counts at iteration 80 {counts.tolist()}, {checked} checked "
          f"({infected_now} newly infected), {time.perf_counter() - t0:.1f} s", flush=True)
    assert checked > 500 and infected_now > 0


def test_large_scale_epidemic_follows_the_sir_equations(abm):
    """At 1.01e7 persons the run is nearly deterministic: the infected share
    of the GPU run follows the SIR equations of Fig 4.17A (peak 0.725 of the
    persons at step 117) as closely as the oracle's small runs do."""
    from scipy.integrate import solve_ivp
    cfg = inputs.scaled_sir(inputs.SIR_MEASLES, 5000)
    pos, st = inputs.sir_population(cfg["n_susceptible"], cfg["n_infected"], cfg["space"], seed=21)
    gp, _ = _params(abm, cfg, 21, space=cfg["space"])
    g = abm.Sir(gp, pos, st, hist_cap=512)
    del pos, st
    h = g.step(400, counts=True)
    n = cfg["n_susceptible"] + cfg["n_infected"]
    b, gam = cfg["beta"], cfg["gamma"]
    y = solve_ivp(lambda _, v: [-b * v[0] * v[1] / n, b * v[0] * v[1] / n - gam * v[1], gam * v[1]], (0, 400),
                  [cfg["n_susceptible"], cfg["n_infected"], 0.0], t_eval=np.arange(1, 401), rtol=1e-10,
                  atol=1e-8).y.T / n
    inf = h[:, 1] / n
    print(f"1.01e7 persons: peak infected {inf.max():.4f} at step {int(inf.argmax()) + 1} (equations "
          f"{y[:, 1].max():.4f} at {int(y[:, 1].argmax()) + 1}), largest gap {np.abs(inf - y[:, 1]).max():.4f}",
          flush=True)
    assert np.all(h.sum(axis=1) == n)
    assert abs(inf.max() - y[:, 1].max()) <= 0.03
    assert abs(int(inf.argmax()) - int(y[:, 1].argmax())) <= 10
    assert np.abs(inf - y[:, 1]).max() <= 0.1


def test_counts_through_a_short_history_ring(abm):
    """A history of 4 iterations returns the counts of a 25-iteration step in
    chunks of 3 (the end of each iteration clears the next slot), equal to
    the counts of a run with a long history and to the oracle's."""
    cfg = inputs.SIR_MEASLES
    pos, st = inputs.sir_population(500, 50, 40.0, seed=6)
    gp, op = _params(abm, cfg, 6, space=40.0)
    short = abm.Sir(gp, pos, st, hist_cap=4)
    long_ = abm.Sir(gp, pos, st, hist_cap=64)
    o = osir.OracleSIR(pos, st, op)
    hs = np.concatenate([short.step(25, counts=True), short.step(7, counts=True)])
    hl = long_.step(32, counts=True)
    assert np.array_equal(hs, hl)
    assert np.array_equal(hs, o.step(32))
    with pytest.raises(abm.AbmError):  # a history needs at least two slots
        abm.Sir(gp, pos, st, hist_cap=1)


def _box_keys(pos, dims, box_len):
    """Linear box of every position (x fastest), by the grid's FP64 division."""
    b = np.clip(np.floor(pos / box_len), 0, dims - 1).astype(np.int64)
    return b[:, 0] + dims * (b[:, 1] + dims * b[:, 2])


def test_persons_are_stored_in_box_order_after_each_person_sort(abm):
    """Results do not depend on the storage order, so a broken person sort
    would only cost speed; this checks the order itself.  Right after
    creation and after the sort that ends every 64th iteration, the box
    keys of the stored persons never decrease, and the persons are the same
    uids as the oracle's with the same states and positions."""
    cfg = dict(inputs.SIR_MEASLES)
    pos, st = inputs.sir_population(6000, 60, 150.0, seed=14)
    gp, op = _params(abm, cfg, 14, space=150.0)
    g = abm.Sir(gp, pos, st, hist_cap=8)
    o = osir.OracleSIR(pos, st, op)
    dims, box_len = g.grid()
    assert dims > 4
    assert np.all(np.diff(_box_keys(g.query(abm.SIR_POS), dims, box_len)) >= 0), "not in box order at creation"
    for k in range(2):
        g.step(64)
        o.step(64)
        keys = _box_keys(g.query(abm.SIR_POS), dims, box_len)
        assert np.all(np.diff(keys) >= 0), f"not in box order after iteration {64 * (k + 1) - 1}"
        _same_state(abm, g, o, f"after {64 * (k + 1)} iterations")
    g.step(5)  # between two sorts the persons drift out of order
    o.step(5)
    _same_state(abm, g, o, "after 133 iterations")
