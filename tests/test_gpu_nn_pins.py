"""Element-wise GPU parity of the learned part's small kernels: the Adam
update, the masked mean squared error with its gradient, and the velocity
output, each against its float64 reference or its definition."""
import numpy as np
import pytest
import torch

from oracle import cnn_oracle as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def NN():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_11468_amd import nn
    nn._lib()
    return nn


def _bits(t):
    """uint16 bit patterns of a bf16 tensor."""
    return t.cpu().view(torch.int16).numpy().view(np.uint16)


@pytest.mark.parametrize("lr,b1,b2", [(1e-3, 0.9, 0.999), (3e-2, 0.8, 0.99)])
def test_adam_step_matches_reference(NN, lr, b1, b2):
    """Five Adam updates (t = 1..5) with fresh gradients of mixed scales.
    Each update from the GPU's own float32 state agrees with the float64
    reference to float32 rounding; the five-step trajectory stays within
    1e-6 (relative max-abs) of the reference trajectory; the bf16 copy is
    the round-to-nearest-even of the float32 master, bit for bit."""
    dev = torch.device("cuda")
    n = 4099  # not a multiple of the workgroup size
    rng = np.random.default_rng(11)
    p0 = rng.normal(size=n).astype(np.float32)
    p = torch.from_numpy(p0).to(dev)
    m = torch.zeros(n, dtype=torch.float32, device=dev)
    v = torch.zeros(n, dtype=torch.float32, device=dev)
    pb = torch.empty(n, dtype=torch.bfloat16, device=dev)
    ref_p, ref_m, ref_v = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    eps = 1e-8
    for t in range(1, 6):
        g = (rng.normal(size=n) * 10.0 ** rng.uniform(-4, 1, size=n)).astype(np.float32)
        before = (p.cpu().numpy().astype(np.float64), m.cpu().numpy().astype(np.float64),
                  v.cpu().numpy().astype(np.float64))
        NN.adam_step(p, torch.from_numpy(g).to(dev), m, v, pb, lr, b1, b2, eps, t)
        torch.cuda.synchronize()
        got_p, got_m, got_v = (x.cpu().numpy().astype(np.float64) for x in (p, m, v))
        # one update from the same (float32) state
        one_p, one_m, one_v = R.adam_step(before[0], g, before[1], before[2], t, lr, b1, b2, eps)
        assert np.abs(got_p - one_p).max() <= 4e-7 * np.abs(one_p).max()
        assert np.abs(got_m - one_m).max() <= 4e-7 * np.abs(one_m).max()
        assert np.abs(got_v - one_v).max() <= 4e-7 * np.abs(one_v).max()
        # the trajectory from the common start
        ref_p, ref_m, ref_v = R.adam_step(ref_p, g, ref_m, ref_v, t, lr, b1, b2, eps)
        for got, ref in ((got_p, ref_p), (got_m, ref_m), (got_v, ref_v)):
            assert np.abs(got - ref).max() <= 1e-6 * np.abs(ref).max(), t
        # the bf16 copy rounds the float32 master to nearest even
        assert np.array_equal(_bits(pb), R.bf16_bits_rne(p.cpu().numpy()))
    # the updates actually moved the parameters by about lr per step
    assert np.abs(ref_p - p0).max() > 2 * lr


@pytest.mark.parametrize("n,solid_frac", [(5000, 0.3), (70001, 0.6)])
def test_masked_mse_loss_and_gradient(NN, n, solid_frac):
    """Loss against autograd in float64 (float32 sums); the bf16 head
    gradient equals the round-to-nearest-even of 2 (pred - target) / (3 Nf)
    computed in float32 (the kernel's precision), bit for bit, and lies
    within one bf16 ulp of the float64 autograd gradient; solid voxels and
    the padding channels 3..15 get exactly zero."""
    dev = torch.device("cuda")
    rng = np.random.default_rng(n)
    pred = rng.normal(size=(n, 3)).astype(np.float32)
    tgt = rng.normal(size=(n, 3)).astype(np.float32)
    solid = rng.uniform(size=n) < solid_frac
    mask = solid.astype(np.uint8)
    dy = torch.empty(n * 16, dtype=torch.bfloat16, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    ws = torch.empty(4096, dtype=torch.float32, device=dev)
    NN.masked_mse(torch.from_numpy(pred).to(dev), torch.from_numpy(tgt).to(dev),
                  torch.from_numpy(mask).to(dev), dy, loss, ws)
    torch.cuda.synchronize()
    pr = torch.from_numpy(pred.astype(np.float64)).requires_grad_()
    L = R.masked_mse(pr, torch.from_numpy(tgt.astype(np.float64)), torch.from_numpy(~solid))
    L.backward()
    assert abs(loss.item() - L.item()) <= 1e-5 * L.item()
    got = _bits(dy).reshape(n, 16)
    assert np.all(got[:, 3:] == 0)
    assert np.all(got[solid, :3] == 0)
    nf = np.float32((~solid).sum())
    g32 = (np.float32(2.0) * (pred - tgt)) / (np.float32(3.0) * nf)
    g32[solid] = 0.0
    assert np.array_equal(got[:, :3], R.bf16_bits_rne(g32))
    as_f = torch.from_numpy(got[:, :3].astype(np.int16)).view(torch.bfloat16).double().numpy()
    ref = pr.grad.numpy()
    assert np.all(np.abs(as_f - ref) <= 2.0 ** -7 * np.abs(ref) + 1e-30)


def test_velocity_out_definition(NN):
    """u[a][i] = scale * pred[i][a] in float64 on fluid voxels, 0 on solid
    voxels, bit for bit."""
    dev = torch.device("cuda")
    n = 12345
    rng = np.random.default_rng(4)
    pred = rng.normal(size=(n, 3)).astype(np.float32)
    mask = (rng.uniform(size=n) < 0.4).astype(np.uint8)
    scale = 1e-5 / 0.1 * 0.0371
    u = torch.full((3 * n,), np.nan, dtype=torch.float64, device=dev)
    NN.velocity_out(torch.from_numpy(pred).to(dev), torch.from_numpy(mask).to(dev), scale, u)
    want = scale * pred.astype(np.float64).T.copy()
    want[:, mask != 0] = 0.0
    assert np.array_equal(u.cpu().numpy().reshape(3, n), want)


@pytest.mark.parametrize("n", [16, 12, 48])
def test_distance_features_closed_form(NN, n):
    """nn_prepare_input_dist around a single solid voxel of a periodic cube:
    the 26-neighbourhood chamfer distance to it has the closed form
    (a - b) + (b - c) sqrt 2 + c sqrt 3 for sorted offsets a >= b >= c
    (minimum image), clamped at dmax; channels 2 and 3 carry d/dmax and
    (d/dmax)^2 rounded to bf16 (within one bf16 ulp of the float64 value,
    since the kernel sums the steps in float32), channels 0/1 the solid and
    fluid indicators, the padding channels zero.  Two cubes in one batch,
    the solid voxel at different places (the batch index does not leak).
    Edges 16 and 48 take the kernel's runs of 8 planes per thread (two and
    six runs per column), 12 the one-plane form; cpad 16 the 8-channel
    stores, cpad 12 the one-channel ones."""
    dev = torch.device("cuda")
    dmax, cpad = 6.0, (12 if n == 12 else 16)
    mask = np.zeros((2, n, n, n), np.uint8)       # [b][z][y][x]
    spots = [(3, 5, 7), (n - 4, 0, n - 1)]        # (x, y, z)
    for b, (x, y, z) in enumerate(spots):
        mask[b, z, y, x] = 1
    x_t = torch.empty(2 * n ** 3 * cpad, dtype=torch.bfloat16, device=dev)
    work = torch.empty(2 * 2 * n ** 3, dtype=torch.float32, device=dev)
    NN.prepare_input_dist(torch.from_numpy(mask.reshape(-1)).to(dev), x_t, 2, n, cpad, dmax, work)
    got = x_t.float().cpu().numpy().reshape(2, n, n, n, cpad)
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    for b, (x0, y0, z0) in enumerate(spots):
        off = [np.minimum(np.abs(v - v0), n - np.abs(v - v0)) for v, v0 in ((xx, x0), (yy, y0), (zz, z0))]
        srt = np.sort(np.stack(off), axis=0)[::-1]
        a, bb, c = srt[0], srt[1], srt[2]
        d = np.minimum((a - bb) + (bb - c) * np.sqrt(2.0) + c * np.sqrt(3.0), dmax)
        q = d / dmax
        solid = mask[b] != 0
        assert np.array_equal(got[b, ..., 0], solid.astype(np.float32))
        assert np.array_equal(got[b, ..., 1], (~solid).astype(np.float32))
        for ch, want in ((2, q), (3, q * q)):
            assert np.all(np.abs(got[b, ..., ch] - want) <= 2.0 ** -8 * np.abs(want) + 1e-30), ch
        assert np.all(got[b, ..., 4:] == 0)
    # the clamp is reached somewhere and the distances are not all equal
    assert got[0, ..., 2].max() == 1.0 and got[0, ..., 2][mask[0] == 0].min() == pytest.approx(1 / dmax, rel=1e-2)


def test_velocity_labels_inverse_of_velocity_out(NN):
    """nn_velocity_labels(u, mask, s) = s * u transposed to [n][3] in
    float32 (round to nearest), 0 on solids; fed back through
    nn_velocity_out with scale 1/s it returns u to float32 precision."""
    dev = torch.device("cuda")
    n = 9999
    rng = np.random.default_rng(6)
    u = rng.normal(size=(3, n)) * 1e-3
    mask = (rng.uniform(size=n) < 0.4).astype(np.uint8)
    u[:, mask != 0] = 0.0
    scale = 1.0 / (1e-6 / 0.1 * 0.37)
    out = torch.full((n * 3,), np.nan, dtype=torch.float32, device=dev)
    m_t = torch.from_numpy(mask).to(dev)
    NN.velocity_labels(torch.from_numpy(u.reshape(-1)).to(dev), m_t, scale, out)
    want = (scale * u).T.astype(np.float32)
    want[mask != 0] = 0.0
    assert np.array_equal(out.cpu().numpy().reshape(n, 3), want)
    back = torch.empty(3 * n, dtype=torch.float64, device=dev)
    NN.velocity_out(out, m_t, 1.0 / scale, back)
    assert np.allclose(back.cpu().numpy().reshape(3, n), u, rtol=2 ** -23, atol=0)
