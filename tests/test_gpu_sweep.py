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
