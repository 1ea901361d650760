"""abm_mlp_infer_noalloc (the forward pass with its activations in the
library's fixed device array) against abm_mlp_infer (activations in the
handle's workspace): the same kernels and arithmetic, so the outputs must be
equal bit for bit.  Two calls in a row, the second with a smaller batch (the
array keeps the first call's contents), and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abm():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2503_10796_amd import abm as _abm
    _abm.lib()
    return _abm


def test_noalloc_inference_equals_workspace_inference(abm):
    import torch
    m = abm.Mlp((35, 256, 256, 256, 32), max_batch=4096, seed=3)
    rng = np.random.default_rng(17)
    for batch in (4096, 777):  # the second call is smaller than the first
        x = torch.as_tensor(rng.normal(size=(batch, 35)).astype(np.float32), device="cuda")
        y_ws = torch.empty((batch, 32), dtype=torch.float32, device="cuda")
        y_na = torch.full((batch, 32), float("nan"), dtype=torch.float32, device="cuda")
        m.infer(x, out=y_ws)
        m.infer_noalloc(x, y_na)
        torch.cuda.synchronize()
        a, b = y_ws.cpu().numpy(), y_na.cpu().numpy()
        assert np.all(np.isfinite(b))
        assert np.array_equal(a, b), f"batch {batch}: max difference {np.abs(a - b).max()}"
    x = torch.zeros((4097, 35), dtype=torch.float32, device="cuda")
    y = torch.zeros((4097, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(abm.AbmError) as e:
        m.infer_noalloc(x, y)
    assert e.value.code == abm.ERR_ARG
