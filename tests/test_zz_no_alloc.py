"""The allocation-free masked MSE (nn_masked_mse_noalloc) against the
workspace entry point it varies (nn_masked_mse): the same loss and the same
bf16 gradient, bit for bit, on two calls in a row, the second with fewer
voxels (so the library's scratch still holds the first call's partials)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def NN():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_11468_amd import nn
    nn._lib()
    return nn


def _case(n, solid_frac, seed, dev):
    rng = np.random.default_rng(seed)
    pred = torch.from_numpy(rng.normal(size=(n, 3)).astype(np.float32)).to(dev)
    tgt = torch.from_numpy(rng.normal(size=(n, 3)).astype(np.float32)).to(dev)
    mask = torch.from_numpy((rng.uniform(size=n) < solid_frac).astype(np.uint8)).to(dev)
    return pred, tgt, mask


def _bits(t):
    return t.cpu().view(torch.int16).numpy()


def test_noalloc_matches_workspace_entry_point(NN):
    dev = torch.device("cuda")
    for n, frac, seed in ((700001, 0.6, 1), (5003, 0.3, 2)):
        pred, tgt, mask = _case(n, frac, seed, dev)
        dy_ref = torch.full((n * 16,), 7.0, dtype=torch.bfloat16, device=dev)
        loss_ref = torch.full((1,), -1.0, dtype=torch.float32, device=dev)
        ws = torch.full((4096,), np.nan, dtype=torch.float32, device=dev)
        NN.masked_mse(pred, tgt, mask, dy_ref, loss_ref, ws)
        dy = torch.full((n * 16,), -3.0, dtype=torch.bfloat16, device=dev)
        loss = torch.full((1,), -2.0, dtype=torch.float32, device=dev)
        NN.masked_mse_noalloc(pred, tgt, mask, dy, loss)
        torch.cuda.synchronize()
        assert loss.item() == loss_ref.item() and loss.item() > 0, (n, loss.item(), loss_ref.item())
        assert np.array_equal(_bits(dy), _bits(dy_ref)), n
        # the loss is the masked mean squared error (float32 sums)
        fl = mask.cpu().numpy() == 0
        d = (pred.cpu().numpy() - tgt.cpu().numpy())[fl].astype(np.float64)
        assert loss.item() == pytest.approx((d ** 2).mean(), rel=1e-5)


def test_noalloc_rejects_oversized_input(NN):
    """More voxels than the documented maximum are refused before any
    launch (the buffers here are tiny; nothing reads past them)."""
    dev = torch.device("cuda")
    pred, tgt, mask = _case(16, 0.5, 3, dev)
    dy = torch.empty(16 * 16, dtype=torch.bfloat16, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    with pytest.raises(RuntimeError, match="exceed the maximum"):
        NN.masked_mse_noalloc(pred, tgt, mask, dy, loss, n=(1 << 31))
