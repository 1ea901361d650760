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
