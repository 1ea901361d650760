"""Batched parameter sweep: one graph launch per iteration for all simulations,
autotuned schedule; results equal those of the per-simulation path."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10796_amd import abm, sweep
    abm.lib()
    return abm, sweep


def test_batched_counts_match_the_lineage_count(mods):
    _, sweep = mods
    cfg = sweep.SweepConfig(24, seed=4, iters=60)
    _, _, n_end, _ = sweep.run_batched(cfg, record=False, tune=True)
    exact = np.array([cfg.counts(s, *cfg.state(s)[2:4])[-1] for s in range(cfg.n_sims)]).astype(np.int64)
    assert np.array_equal(n_end, exact)


def test_autotuned_batch_equals_per_simulation_runs(mods):
    """The tuner times candidate schedules from a snapshot and restores it;
    the tuned batch then matches each simulation run on its own, bitwise."""
    abm, sweep = mods
    cfg = sweep.SweepConfig(12, seed=4, iters=40, n_hi=4000.0)
    b, states, caps = sweep.build_batch(cfg)
    b.tune(2)
    b.step(cfg.iters)
    for s in range(cfg.n_sims):
        pos, diam, vol, growth = states[s]
        p = abm.Population(cfg.params(s), pos, diam, vol=vol, growth=growth, capacity=caps[s],
                           box_capacity=3 * caps[s] + 65536)
        p.step(cfg.iters)
        ub, us = b.query(abm.UID, s), p.query(abm.UID)
        assert np.array_equal(np.sort(ub), np.sort(us))
        assert np.array_equal(b.query(abm.POS, s)[np.argsort(ub)], p.query(abm.POS)[np.argsort(us)])
        assert np.array_equal(b.query(abm.VOL, s)[np.argsort(ub)], p.query(abm.VOL)[np.argsort(us)])
        p.close()


def test_histograms_match_the_oracle_statistics(mods):
    abm, sweep = mods
    from oracle import sim as osim
    cfg = sweep.SweepConfig(6, seed=4, iters=20, n_hi=3000.0)
    b, states, _ = sweep.build_batch(cfg)
    b.step(cfg.iters)
    c, rg, rm, h = b.stats(sweep.HIST_RMAX)
    for s in range(cfg.n_sims):
        pos = b.query(abm.POS, s)
        oc, org, orm, oh, _ = osim.stats(pos, sweep.HIST_RMAX)
        assert np.allclose(c[s], oc, rtol=0, atol=1e-12)
        assert rg[s] == pytest.approx(org, rel=1e-13)
        assert np.allclose(h[s], oh, rtol=1e-6)


def test_tuned_batch_extremes_match_the_oracle(mods):
    """Simulations of the seed-4 sweep at its extremes -- division diameters
    near 6 um (burst divisions at the start, about 70 agents per box), the
    lowest and highest adherence, the fastest growth -- in one tuned batch in
    the sweep's launch configuration (static skip, re-sort every 10).  At
    iterations 0, 1, 2 (divisions), 10 (after a re-sort) and 30 every
    simulation is stepped once by the oracle from its GPU state and compared
    agent by agent: same agents, volumes and diameters bit for bit, contact
    and non-zero-force counts exact, forces within 1e-5 of the sum of |F_N|,
    move decisions, positions and static flags (Algorithm 2, Eq 4.1-4.2)."""
    abm, sweep = mods
    from tests import helpers as H
    cfg = sweep.SweepConfig(256, seed=4, iters=41)  # capacities for 31 + 10 iterations
    sims = [73, 24, 218, 201, 148, 143]  # d_div 6.04 / 6.08, adherence 0.904 / 2.689 / 2.695, growth scale 1.5
    b, states, caps = sweep.build_batch(cfg, sims, record=True)
    b.tune(2)
    checks = {0, 1, 2, 10, 30}
    for it in range(31):
        if it not in checks:
            b.step(1)
            continue
        snaps = [H.gpu_state(abm, b, k) for k in range(len(sims))]
        b.step(1)
        for k, s in enumerate(sims):
            st = snaps[k]
            op = H.oracle_params(box_len=0.0, div_vol=sweep.inputs.division_volume(float(cfg.d_div[s])),
                                 adherence=float(cfg.adherence[s]), detect_static=True, seed=cfg.seed, sim_id=s)
            nu = int(st["uid"].max()) + 1
            o = H.oracle_from_state(st, op, cap=caps[k], next_uid=nu, iteration=it)
            o.step(1)
            ug = b.query(abm.UID, k)
            og, oo = np.argsort(ug), np.argsort(o.uid[:o.n])
            assert np.array_equal(ug[og], o.uid[:o.n][oo]), (s, it)
            assert np.array_equal(b.query(abm.VOL, k)[og], o.vol[:o.n][oo]), (s, it)
            assert np.array_equal(b.query(abm.DIAM, k)[og], o.diam[:o.n][oo]), (s, it)
            res = H.compare_single_step(abm, b, o, sim=k, check_static=True, check_nbr=False)
            print(f"sim {s} iteration {it}: {o.n} agents, {res}", flush=True)
    # 10-iteration trajectories from iteration 31 (divisions, static skip and a re-sort in between)
    snaps = [H.gpu_state(abm, b, k) for k in range(len(sims))]
    b.step(10)
    for k, s in enumerate(sims):
        st = snaps[k]
        op = H.oracle_params(box_len=0.0, div_vol=sweep.inputs.division_volume(float(cfg.d_div[s])),
                             adherence=float(cfg.adherence[s]), detect_static=True, seed=cfg.seed, sim_id=s)
        o = H.oracle_from_state(st, op, cap=caps[k], next_uid=int(st["uid"].max()) + 1, iteration=31)
        o.step(10)
        ug = b.query(abm.UID, k)
        og, oo = np.argsort(ug), np.argsort(o.uid[: o.n])
        assert np.array_equal(ug[og], o.uid[: o.n][oo]), s
        assert np.array_equal(b.query(abm.VOL, k)[og], o.vol[: o.n][oo]), s
        err = np.linalg.norm(b.query(abm.POS, k)[og] - o.pos()[oo], axis=1)
        print(f"sim {s}: 10-iteration trajectory, {o.n} agents, max {err.max():.3e} um, "
              f"rms {np.sqrt((err ** 2).mean()):.3e} um", flush=True)
        assert err.max() <= 1e-4


def test_tuner_picks_every_schedule_parameter(mods):
    """The tuner picks the unit-sweep work groups, the box-wise work groups
    and waves per work group, and (when asked with a negative period) the
    re-sort period from its candidate sets, and leaves the state unchanged."""
    abm, sweep = mods
    cfg = sweep.SweepConfig(256, seed=4, iters=12)
    sims = [73, 24, 5, 6, 7, 8]
    b, _, _ = sweep.build_batch(cfg, sims, resort_every=-1)
    ref, _, _ = sweep.build_batch(cfg, sims, resort_every=10)
    b.tune(2)
    sc = b.schedule()
    print(sc, flush=True)
    assert sc["sweep_grid"] in (512, 1024, 2048, 4096)
    assert (sc["dense_grid"], sc["dense_waves"]) in ((512, 4), (1024, 4), (2048, 4), (1024, 2), (2048, 2), (4096, 2))
    assert sc["resort_every"] in (5, 10, 20)
    b.step(cfg.iters)
    ref.step(cfg.iters)
    for k in range(len(sims)):
        ub, ur = b.query(abm.UID, k), ref.query(abm.UID, k)
        assert np.array_equal(np.sort(ub), np.sort(ur))
        assert np.array_equal(b.query(abm.POS, k)[np.argsort(ub)], ref.query(abm.POS, k)[np.argsort(ur)])
