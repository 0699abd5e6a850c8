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
