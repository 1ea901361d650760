"""Surrogate screening of parameter sweeps.

An MLP (the library's BF16 matrix-core kernels) maps [3 sweep parameters
scaled to [0, 1], log(1 + radial density histogram at iteration t)] to the
change of log(1 + histogram) from t to t + 50 (so that "no change" is the
zero output).  Training windows come from a batched sweep;
the error is judged against the plain simulation of held-out parameter sets,
next to two references without learning: persistence (the histogram does not
change) and a least-squares linear map of the same inputs.
"""
import time

import numpy as np

from . import abm, sweep

HORIZON = 50
DIMS = (35, 256, 256, 256, 32)


def windows(cfg, hist, n, seed, t_max=250, early=0.0):
    """n training windows (x, y) from histories hist [iters+1, n_sims, 32]:
    t uniform in [0, t_max], or with `early` > 0 that share of the windows
    drawn with density falling as 1/sqrt(t) (more windows near the start,
    where screening begins)."""
    rng = np.random.default_rng(seed)
    s = rng.integers(0, cfg.n_sims, size=n)
    t = rng.integers(0, t_max + 1, size=n)
    k = int(early * n)
    if k:
        t[:k] = np.floor((t_max + 1) * rng.random(k) ** 2).astype(t.dtype)
    x = np.concatenate([cfg.params_unit[s], np.log1p(hist[t, s])], axis=1).astype(np.float32)
    y = (np.log1p(hist[t + HORIZON, s]) - np.log1p(hist[t, s])).astype(np.float32)
    return x, y


def to_hist(x, out, lim=8.0):
    """Histogram predicted from the inputs x and a predicted change of
    log(1 + density), the change clamped to [-lim, lim]."""
    return np.maximum(np.expm1(x[:, 3:].astype(np.float64) + np.clip(out, -lim, lim)), 0.0)


def judge(pred, true, h0, changing=0.1):
    """Relative L2 errors of a prediction next to persistence: median and mean
    over all windows, and median over the windows whose histogram changes by
    more than `changing` (where screening needs a model)."""
    e, ep = rel_err(pred, true), rel_err(h0, true)
    big = ep > changing
    return {"median": float(np.median(e)), "mean": float(np.mean(e)),
            "median_changing": float(np.median(e[big])) if big.any() else None,
            "changing_windows": int(big.sum()), "windows": int(e.size)}


def eval_windows(cfg, hist, times):
    """All (simulation, t) windows at the given times."""
    xs, ys, h0 = [], [], []
    for t in times:
        xs.append(np.concatenate([cfg.params_unit, np.log1p(hist[t])], axis=1))
        ys.append(hist[t + HORIZON])
        h0.append(hist[t])
    return (np.concatenate(xs).astype(np.float32), np.concatenate(ys).astype(np.float64),
            np.concatenate(h0).astype(np.float64))


def shell_r2(rmax=sweep.HIST_RMAX):
    """Mean r^2 over each of the 32 shells and their volumes (um^3)."""
    w = rmax / 32.0
    r0 = w * np.arange(32)
    r1 = r0 + w
    vol = 4.0 / 3.0 * np.pi * (r1 ** 3 - r0 ** 3)
    r2 = 3.0 / 5.0 * (r1 ** 5 - r0 ** 5) / (r1 ** 3 - r0 ** 3)
    return r2, vol


def r_gyr_from_hist(h):
    """Radius of gyration implied by a density histogram (agents per 1000 um^3)."""
    r2, vol = shell_r2()
    n = h * vol / 1000.0
    return np.sqrt((n * r2).sum(axis=1) / np.maximum(n.sum(axis=1), 1e-30))


def rel_err(pred, true):
    return np.linalg.norm(pred - true, axis=1) / np.maximum(np.linalg.norm(true, axis=1), 1e-30)


class Surrogate:
    """The trained network with the scaling of its inputs and outputs (fitted
    on the training windows)."""

    def __init__(self, model, xm, xs, ym, ys):
        self.model, self.xm, self.xs, self.ym, self.ys = model, xm, xs, ym, ys

    def predict_change(self, x):
        import torch
        xn = torch.as_tensor(((x - self.xm) / self.xs).astype(np.float32), device="cuda")
        return self.model.infer(xn).cpu().numpy().astype(np.float64) * self.ys + self.ym

    def predict(self, x):
        return to_hist(x, self.predict_change(x))


def input_scaling(x):
    """Parameters are already in [0, 1]; the 32 histogram inputs share one
    mean and scale, so bins that are rarely occupied in training are not
    amplified."""
    m = np.concatenate([np.full(3, 0.5), np.full(x.shape[1] - 3, x[:, 3:].mean())])
    s = np.concatenate([np.full(3, 0.29), np.full(x.shape[1] - 3, max(x[:, 3:].std(), 1e-6))])
    return m, s


def output_scaling(y):
    """Per-bin mean and scale of the change, the scale floored at a tenth of
    the overall one (bins that hardly change keep a near-zero output)."""
    m = y.mean(axis=0).astype(np.float64)
    s = np.maximum(y.std(axis=0), 0.1 * y.std()).astype(np.float64)
    return m, s


def train(x, y, steps=3000, batch=512, lr=1e-3, seed=0, log=None):
    """Adam on the standardised windows (cosine learning-rate decay); returns
    (Surrogate, seconds)."""
    m = abm.Mlp(DIMS, max_batch=max(batch, 4096), seed=seed)
    rng = np.random.default_rng(seed)
    import torch
    xm, xs = input_scaling(x)
    ym, ys = output_scaling(y)
    xd = torch.as_tensor(((x - xm) / xs).astype(np.float32), device="cuda")
    yd = torch.as_tensor(((y - ym) / ys).astype(np.float32), device="cuda")
    t0 = time.perf_counter()
    loss = None
    for it in range(steps):
        idx = torch.as_tensor(rng.integers(0, x.shape[0], size=batch), device="cuda")
        cos_lr = lr * 0.5 * (1.0 + np.cos(np.pi * it / steps))
        want = (it % 500 == 0) or it == steps - 1
        loss = m.train_step(xd[idx], yd[idx], lr=max(cos_lr, 1e-5), want_loss=want) if want else \
            m.train_step(xd[idx], yd[idx], lr=max(cos_lr, 1e-5), want_loss=False)
        if want and log:
            log(f"[surrogate] step {it} loss {loss:.5f}")
    torch.cuda.synchronize()
    return Surrogate(m, xm, xs, ym, ys), time.perf_counter() - t0


class Linear:
    """Least-squares affine map of the same inputs to the same target (the
    change of log(1 + histogram)); its predictions are clipped per bin to
    the range of changes seen in training, so that it cannot extrapolate
    outside the data it was fitted on."""

    def __init__(self, x, y):
        X = np.concatenate([x.astype(np.float64), np.ones((x.shape[0], 1))], axis=1)
        self.W, *_ = np.linalg.lstsq(X, y.astype(np.float64), rcond=None)
        self.lo, self.hi = y.min(axis=0).astype(np.float64), y.max(axis=0).astype(np.float64)

    def predict_change(self, x):
        X = np.concatenate([x.astype(np.float64), np.ones((x.shape[0], 1))], axis=1)
        return np.clip(X @ self.W, self.lo, self.hi)

    def predict(self, x):
        return to_hist(x, self.predict_change(x))


def predicted_change(x, pred):
    """Relative L2 change of the histogram from the input to the prediction:
    the screen's flag for a fallback (the surrogate is least accurate where
    the spheroid changes most)."""
    h0 = np.expm1(x[:, 3:].astype(np.float64))
    return rel_err(pred, h0)


def pick_threshold(change, err, target):
    """The largest threshold on the predicted change at which the mean error
    over all sets stays within target, when every set above the threshold is
    simulated instead (error 0).  Returns (threshold, fallback fraction)."""
    order = np.argsort(change)
    n = change.size
    kept_err = np.cumsum(err[order])  # error sum if the first k sets keep their prediction
    best_k = 0
    for k in range(1, n + 1):
        if kept_err[k - 1] / n <= target:
            best_k = k
    tau = change[order[best_k - 1]] if best_k > 0 else -1.0
    return float(tau), 1.0 - best_k / n
