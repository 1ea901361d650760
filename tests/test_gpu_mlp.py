"""GPU surrogate MLP (BF16 matrix-core kernels through the C ABI) against the FP64 oracle.

Tolerances: the GEMM operands are rounded to BF16 (unit roundoff 2^-9) and
accumulated in FP32, so each layer's output carries a relative error of a few
2^-9 that partly averages out over the 256-term sums.  The parity bar for the
gradients is per tensor at most 2e-2 normwise relative with cosine at least
0.999, and the forward pass at most 2e-2 normwise (measured: 2-6e-3).
"""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
DIMS = omlp.DIMS


@pytest.fixture(scope="module")
def abm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10796_amd import abm as _abm
    _abm.lib()
    return _abm


def he_theta(seed):
    rng = np.random.default_rng(seed)
    layers = []
    for i in range(len(DIMS) - 1):
        fi, fo = DIMS[i], DIMS[i + 1]
        layers.append((rng.normal(0.0, np.sqrt(2.0 / fi), size=(fo, fi)), rng.normal(0.0, 0.05, size=fo)))
    return omlp.flatten(layers).astype(np.float32).astype(np.float64)


def batch(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.normal(0.0, 1.0, size=(n, DIMS[0])).astype(np.float32)
    y = rng.normal(0.0, 1.0, size=(n, DIMS[-1])).astype(np.float32)
    return x, y


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def cosine(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("n", [1, 64, 300, 4096])
def test_forward_matches_oracle(abm, n):
    m = abm.Mlp(DIMS, max_batch=4096, seed=1)
    theta = he_theta(2)
    m.set_params(theta)
    x, _ = batch(3, n)
    yg = m.infer(x).cpu().numpy().astype(np.float64)
    yo, _ = omlp.forward(theta, x.astype(np.float64))
    e = rel(yg, yo)
    print(f"batch {n}: forward normwise relative error {e:.3e}", flush=True)
    assert e < 2e-2


@pytest.mark.parametrize("n", [37, 256, 1024])
def test_gradients_match_oracle(abm, n):
    m = abm.Mlp(DIMS, max_batch=4096, seed=1)
    theta = he_theta(4)
    m.set_params(theta)
    x, y = batch(5, n)
    lg, g = m.grads(x, y)
    g = g.cpu().numpy().astype(np.float64)
    lo, go = omlp.grads(theta, x.astype(np.float64), y.astype(np.float64))
    assert abs(lg - lo) <= 2e-2 * lo
    gl = omlp.unflatten(g)
    ol = omlp.unflatten(go)
    for li, ((gW, gb), (oW, ob)) in enumerate(zip(gl, ol)):
        eW, eb = rel(gW, oW), rel(gb, ob)
        cW = cosine(gW.ravel(), oW.ravel())
        print(f"batch {n} layer {li}: dW rel {eW:.3e} cos {cW:.6f}, db rel {eb:.3e}", flush=True)
        cb = cosine(gb, ob)
        assert eW <= 2e-2 and eb <= 2e-2 and cW >= 0.999 and cb >= 0.999
    assert cosine(g, go) > 0.999


def test_gradients_are_deterministic(abm):
    m = abm.Mlp(DIMS, max_batch=512, seed=7)
    x, y = batch(8, 512)
    _, g1 = m.grads(x, y)
    _, g2 = m.grads(x, y)
    assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy())


def test_adam_step_matches_oracle_update(abm):
    """One train step = the GPU gradient fed to Adam (bias-corrected) in FP64."""
    m = abm.Mlp(DIMS, max_batch=512, seed=9)
    theta = he_theta(10)
    m.set_params(theta)
    x, y = batch(11, 200)
    _, g = m.grads(x, y)
    g = g.cpu().numpy().astype(np.float64)
    m.train_step(x, y, lr=1e-3)
    new = m.get_params().cpu().numpy().astype(np.float64)
    opt = omlp.Adam(theta.astype(np.float32).astype(np.float64), lr=1e-3)
    ref = opt.step(g)
    step = ref - theta
    assert np.abs(new - ref).max() <= 1e-6 + 1e-3 * np.abs(step).max()


def test_training_reduces_loss(abm):
    """A smooth target the network can fit: the loss falls by 10x in 400 steps."""
    rng = np.random.default_rng(12)
    A = rng.normal(0.0, 1.0 / np.sqrt(DIMS[0]), size=(DIMS[-1], DIMS[0]))
    x = rng.normal(0.0, 1.0, size=(2048, DIMS[0])).astype(np.float32)
    y = np.tanh(x @ A.T).astype(np.float32)
    m = abm.Mlp(DIMS, max_batch=2048, seed=13)
    first = None
    for it in range(400):
        s = (it * 256) % 2048
        loss = m.train_step(x[s:s + 256], y[s:s + 256], lr=1e-3)
        first = loss if first is None else first
    final = np.mean((m.infer(x).cpu().numpy() - y) ** 2)
    print(f"loss {first:.4f} -> {final:.5f}", flush=True)
    assert final < 0.1 * first


def test_error_paths(abm):
    m = abm.Mlp(DIMS, max_batch=64, seed=0)
    x, y = batch(0, 65)
    with pytest.raises(abm.AbmError):
        m.infer(x)
    with pytest.raises(abm.AbmError):
        m.set_params(np.zeros(m.n_params + 1, dtype=np.float32))
    with pytest.raises(abm.AbmError):
        abm.Mlp((35, 250, 32), max_batch=8)  # hidden width not a multiple of 16
