"""The surrogate (trained by the library's own BF16 kernels on windows of a
batched sweep) against the method without it: persistence of the current
histogram, judged on held-out parameter sets by the plain simulation."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10796_amd import abm, sweep, surrogate
    abm.lib()
    return sweep, surrogate


def test_surrogate_beats_persistence_on_held_out_sets(mods):
    sweep, surrogate = mods
    iters = 150
    cfg = sweep.SweepConfig(128, seed=4, iters=iters)
    hist, _, n_end, _ = sweep.run_batched(cfg, record=True, tune=False)
    x, y = surrogate.windows(cfg, hist, 8000, seed=6, t_max=iters - surrogate.HORIZON)
    model, _ = surrogate.train(x, y, steps=2000)
    held = sweep.SweepConfig(128, seed=5, iters=iters)
    hh, _, _, _ = sweep.run_batched(held, record=True, tune=False)
    xe, ye, h0 = surrogate.eval_windows(held, hh, [0, 50, 100])
    j = surrogate.judge(model.predict(xe), ye, h0)
    jp = surrogate.judge(h0, ye, h0)
    print(f"surrogate {j}\npersistence {jp}", flush=True)
    assert j["mean"] < jp["mean"]
    assert j["median_changing"] < 0.7 * jp["median_changing"]


def test_screen_with_simulation_fallback(mods):
    """The screen: sets whose predicted change exceeds a threshold (picked on
    the first half to keep the mean error within 2 %) are simulated instead;
    on the second half the fallback histograms equal the full simulation bit
    for bit and the screened mean error meets the target within a margin."""
    sweep, surrogate = mods
    iters = 100
    cfg = sweep.SweepConfig(128, seed=4, iters=iters)
    hist, _, _, _ = sweep.run_batched(cfg, record=True, tune=False)
    x, y = surrogate.windows(cfg, hist, 8000, seed=6, t_max=iters - surrogate.HORIZON)
    model, _ = surrogate.train(x, y, steps=2000)
    held = sweep.SweepConfig(128, seed=5, iters=surrogate.HORIZON)
    hh, _, _, _ = sweep.run_batched(held, record=True, tune=False)
    xe = np.concatenate([held.params_unit, np.log1p(hh[0])], axis=1).astype(np.float32)
    pred = model.predict(xe)
    change = surrogate.predicted_change(xe, pred)
    err = surrogate.rel_err(pred, hh[surrogate.HORIZON])
    tau, frac = surrogate.pick_threshold(change[:64], err[:64], 0.02)
    flag = np.nonzero(change[64:] > tau)[0] + 64
    final = pred[64:].copy()
    if flag.size:
        hf, _, _, _ = sweep.run_batched(held, record=True, tune=False, sims=list(flag), iters=surrogate.HORIZON)
        assert np.array_equal(hf[surrogate.HORIZON], hh[surrogate.HORIZON][flag])
        final[flag - 64] = hf[surrogate.HORIZON]
    e = surrogate.rel_err(final, hh[surrogate.HORIZON][64:])
    print(f"threshold {tau:.4f}, fallback {flag.size} of 64 (pick half {frac:.2f}), mean error {e.mean():.4f} "
          f"(surrogate alone {err[64:].mean():.4f})", flush=True)
    assert e.mean() < 0.04 and flag.size < 64
