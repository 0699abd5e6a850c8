"""Pins of the CPU float64 network reference: autograd gradients agree with
central finite differences (so the reference differentiates the function
it claims to), and the circular convolution matches a direct loop."""
import numpy as np
import pytest
import torch

from oracle import cnn_oracle as R


def test_conv_matches_direct_sum():
    """3x3x3 circular convolution, stride 1 and 2, against an explicit loop
    over taps with periodic indices."""
    g = torch.Generator().manual_seed(0)
    x = torch.randn(1, 6, 4, 8, 3, generator=g, dtype=torch.float64)
    w = torch.randn(27, 2, 3, generator=g, dtype=torch.float64)
    b = torch.randn(2, generator=g, dtype=torch.float64)
    for stride in (1, 2):
        y = R.conv(x, w, b, stride=stride, act=False)
        D, H, W = 6 // stride, 4 // stride, 8 // stride
        assert y.shape == (1, D, H, W, 2)
        for (z, yy, xx) in [(0, 0, 0), (D - 1, H - 1, W - 1), (1, 0, 2)]:
            acc = b.clone()
            for t in range(27):
                dz, dy, dx = t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1
                v = x[0, (stride * z + dz) % 6, (stride * yy + dy) % 4, (stride * xx + dx) % 8]
                acc = acc + w[t] @ v
            assert torch.allclose(y[0, z, yy, xx], acc, rtol=1e-13, atol=1e-13)


def _tiny_params(seed):
    g = torch.Generator().manual_seed(seed)
    shapes = {"e0a": (27, 16, 16), "e0": (27, 16, 16), "d1": (27, 32, 16), "e1a": (27, 32, 32),
              "e1": (27, 32, 32), "d2": (27, 64, 32), "e2a": (27, 64, 64), "e2": (27, 64, 64),
              "d3": (27, 64, 64), "e3a": (27, 64, 64), "e3": (27, 64, 64), "u2a": (27, 64, 128),
              "u2": (27, 64, 64), "u1a": (27, 32, 96), "u1": (27, 32, 32), "u0a": (27, 16, 48),
              "u0": (27, 16, 16), "head": (1, 16, 16)}
    p = {}
    for k, s in shapes.items():
        w = torch.randn(*s, generator=g, dtype=torch.float64) * (2.0 / (s[0] * s[2])) ** 0.5
        p[k] = (w.requires_grad_(), (0.01 * torch.randn(s[1], generator=g, dtype=torch.float64)).requires_grad_())
    return p


def test_unet_gradient_finite_differences():
    """Autograd gradient of the masked MSE of the reference U-Net equals
    central finite differences (relative error < 1e-6) for sampled weights
    of several layers."""
    torch.manual_seed(0)
    n = 8
    p = _tiny_params(1)
    g = torch.Generator().manual_seed(2)
    solid = (torch.rand(1, n, n, n, generator=g) < 0.3)
    x = torch.zeros(1, n, n, n, 16, dtype=torch.float64)
    x[..., 0] = solid.double()
    x[..., 1] = (~solid).double()
    tgt = torch.randn(1, n, n, n, 3, generator=g, dtype=torch.float64)
    fluid = ~solid

    def loss_fn():
        return R.masked_mse(R.unet(x, p), tgt, fluid)

    loss = loss_fn()
    loss.backward()
    rng = np.random.default_rng(3)
    for name in ("e0a", "d2", "e3", "u1a", "head"):
        w, b = p[name]
        for _ in range(3):
            idx = tuple(int(rng.integers(0, s)) for s in w.shape)
            if name == "head":
                idx = (0, int(rng.integers(0, 3)), idx[2])
            h = 1e-6
            with torch.no_grad():
                w[idx] += h
                lp = loss_fn().item()
                w[idx] -= 2 * h
                lm = loss_fn().item()
                w[idx] += h
            fd = (lp - lm) / (2 * h)
            ad = w.grad[idx].item()
            assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3), (name, idx, fd, ad)


def test_adam_first_step_closed_form():
    """From zero moments the first update is -lr g / (|g| + eps): the bias
    corrections undo the (1 - beta) factors exactly."""
    rng = np.random.default_rng(0)
    p = rng.normal(size=50)
    g = rng.normal(size=50) * 10.0 ** rng.uniform(-6, 2, size=50)
    out, m, v = R.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    np.testing.assert_allclose(out - p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-13)


def test_adam_constant_gradient_every_step():
    """With a constant gradient the bias-corrected moments equal g and g^2
    at every step, so every update is -lr g / (|g| + eps)."""
    g = np.array([2.0, -0.5, 1e-3, -7.0])
    p = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 8):
        new, m, v = R.adam_step(p, g, m, v, t, lr=0.01, beta1=0.8, beta2=0.99)
        np.testing.assert_allclose(new - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        p = new


def test_adam_matches_torch_optimizer():
    """Five updates with changing gradients agree with torch.optim.Adam
    (float64, CPU), an independent implementation of the same algorithm."""
    rng = np.random.default_rng(1)
    p0 = rng.normal(size=64)
    grads = [rng.normal(size=64) * s for s in (1.0, 0.3, 3.0, 1e-3, 0.5)]
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=2e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(64), np.zeros(64)
    for t, g in enumerate(grads, start=1):
        w.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = R.adam_step(p, g, m, v, t, lr=2e-3)
        np.testing.assert_allclose(p, w.detach().numpy(), rtol=1e-14, atol=1e-16)


def test_bf16_rounding_bits():
    """The integer round-to-nearest-even to bf16 agrees with torch's
    conversion, including exact ties, and keeps exactly representable
    values."""
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 3.1415926, -2.5e-7,
                     1.0 + 2 ** -7, 65504.0, 1e30], dtype=np.float32)
    rng = np.random.default_rng(5)
    vals = np.concatenate([vals, rng.normal(size=1000).astype(np.float32) * 10.0])
    want = torch.from_numpy(vals).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(R.bf16_bits_rne(vals), want)
    # ties go to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert R.bf16_bits_rne(np.float32(1.0 + 2 ** -8)) == 0x3F80
    assert R.bf16_bits_rne(np.float32(1.0 + 3 * 2 ** -8)) == 0x3F82


def test_chamfer_distance_brute_force():
    """The reference distance features: for the 26-neighbourhood with step
    lengths 1, sqrt 2, sqrt 3 the shortest path between two voxels with
    sorted offsets a >= b >= c is (a - b) + (b - c) sqrt 2 + c sqrt 3, so
    the distance to the nearest solid is the minimum of that closed form
    over the solid voxels (periodic minimum image): brute force on small
    random boxes, and the clamp."""
    import numpy as np
    rng = np.random.default_rng(9)
    solid = rng.uniform(size=(2, 6, 7, 5)) < 0.08
    solid[1, 0, 0, 0] = True
    got = R.chamfer_distance(solid, 100.0)
    for b in range(2):
        D, H, W = solid[b].shape
        pts = np.argwhere(solid[b])
        for z in range(D):
            for y in range(H):
                for x in range(W):
                    best = np.inf
                    for (pz, py, px) in pts:
                        off = sorted([min(abs(x - px), W - abs(x - px)), min(abs(y - py), H - abs(y - py)),
                                      min(abs(z - pz), D - abs(z - pz))], reverse=True)
                        a, bb, c = off
                        best = min(best, (a - bb) + (bb - c) * np.sqrt(2) + c * np.sqrt(3))
                    assert abs(got[b, z, y, x] - best) <= 1e-12
    clamped = R.chamfer_distance(solid, 1.5)
    assert clamped.max() == 1.5 and np.all(clamped[solid] == 0)
