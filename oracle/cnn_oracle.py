"""CPU float64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

Plain PyTorch CPU operations in float64: ``conv3d`` on circularly padded
input, leaky ReLU, nearest-neighbour upsampling, concatenation, masked mean
squared error, with gradients from autograd; the Adam update written out
from its definition (Kingma and Ba, "Adam: A Method for Stochastic
Optimization", 2015, Algorithm 1) in float64 numpy; the network's distance
input features from a library shortest-path routine (scipy's Dijkstra) on
the voxel graph.  It shares no code with the
GPU kernels; it takes the same weights (rounded to bf16 by the caller when
comparing with the bf16 kernels) in the layout [taps][c_out][c_in] and
channels-last activations [B][D][H][W][C].
"""
from __future__ import annotations

import torch
import torch.nn.functional as F

SLOPE = 0.1
CH = (16, 32, 64, 64)


def to_ncdhw(x):
    return x.permute(0, 4, 1, 2, 3)


def to_ndhwc(x):
    return x.permute(0, 2, 3, 4, 1)


def conv(x, w, b, stride=1, taps=27, act=True, slope=SLOPE):
    """x: [B,D,H,W,Ci]; w: [taps][Co][Ci]; b: [Co] or None -> [B,D',H',W',Co]."""
    co, ci = w.shape[1], w.shape[2]
    xt = to_ncdhw(x)
    if taps == 27:
        wt = w.reshape(3, 3, 3, co, ci).permute(3, 4, 0, 1, 2)
        y = F.conv3d(F.pad(xt, (1, 1, 1, 1, 1, 1), mode="circular"), wt, b, stride=stride)
    else:
        y = F.conv3d(xt, w.reshape(co, ci, 1, 1, 1), b)
    if act:
        y = F.leaky_relu(y, slope)
    return to_ndhwc(y)


def up_concat(coarse, skip):
    up = to_ndhwc(F.interpolate(to_ncdhw(coarse), scale_factor=2, mode="nearest"))
    return torch.cat([up, skip], dim=-1)


def unet(x, params):
    """params: dict name -> (w, b) float64 tensors, names as in the GPU net."""
    def c(name, t, **kw):
        w, b = params[name]
        return conv(t, w, b, **kw)
    e0 = c("e0", c("e0a", x))
    e1 = c("e1", c("e1a", c("d1", e0, stride=2)))
    e2 = c("e2", c("e2a", c("d2", e1, stride=2)))
    e3 = c("e3", c("e3a", c("d3", e2, stride=2)))
    u2 = c("u2", c("u2a", up_concat(e3, e2)))
    u1 = c("u1", c("u1a", up_concat(u2, e1)))
    u0 = c("u0", c("u0a", up_concat(u1, e0)))
    return c("head", u0, taps=1, act=False)[..., :3]


def masked_mse(pred, target, fluid):
    """Mean over fluid voxels and the 3 components of (pred - target)^2."""
    d = (pred - target)[fluid]
    return (d * d).sum() / (3.0 * fluid.sum())


def bf16_round(t):
    """Round float64 values to bf16 (round to nearest even) and back."""
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def adam_step(param, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in float64 (Kingma and Ba, Algorithm 1): the biased
    first and second moment estimates m <- beta1 m + (1 - beta1) g and
    v <- beta2 v + (1 - beta2) g^2, their bias corrections
    m_hat = m / (1 - beta1^t) and v_hat = v / (1 - beta2^t), and the step
    param <- param - lr m_hat / (sqrt(v_hat) + eps).  t >= 1 is the index of
    this update.  Returns (param, m, v) as new float64 arrays."""
    import numpy as np
    p = np.asarray(param, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m_new = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v_new = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m_new / (1.0 - beta1 ** t)
    v_hat = v_new / (1.0 - beta2 ** t)
    return p - lr * m_hat / (np.sqrt(v_hat) + eps), m_new, v_new


def bf16_bits_rne(x):
    """bfloat16 bit patterns (uint16) of float32 values, round to nearest
    even, by integer arithmetic on the float32 bits (finite inputs)."""
    import numpy as np
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def chamfer_distance(solid, dmax):
    """Distance of every voxel of the periodic boxes ``solid`` (bool
    [B][D][H][W]) to the nearest solid voxel along paths of the
    26-neighbourhood with step lengths 1, sqrt 2 and sqrt 3 (the 3-D
    chamfer metric of Borgefors, "Distance transformations in digital
    images", 1986, with exact step lengths), clamped at dmax.  Computed as
    shortest paths from a virtual source joined to every solid voxel
    (scipy.sparse.csgraph.dijkstra), float64 [B][D][H][W]."""
    import numpy as np
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import dijkstra
    solid = np.asarray(solid, dtype=bool)
    out = np.empty(solid.shape)
    for b in range(solid.shape[0]):
        D, H, W = solid[b].shape
        n = D * H * W
        z, y, x = np.meshgrid(np.arange(D), np.arange(H), np.arange(W), indexing="ij")
        idx = (z * H + y) * W + x
        rows, cols, vals = [], [], []
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    k = dz * dz + dy * dy + dx * dx
                    if k == 0:
                        continue
                    nb = (((z + dz) % D) * H + (y + dy) % H) * W + (x + dx) % W
                    rows.append(idx.ravel())
                    cols.append(nb.ravel())
                    vals.append(np.full(n, np.sqrt(k)))
        src = np.flatnonzero(solid[b].ravel())
        rows.append(np.full(src.size, n))
        cols.append(src)
        vals.append(np.full(src.size, 1e-300))  # virtual source, zero length in effect
        g = coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(n + 1, n + 1)).tocsr()
        d = dijkstra(g, directed=True, indices=n)[:n]
        d[solid[b].ravel()] = 0.0  # (the virtual edges carry a tiny length,
        #                             since the graph routine drops zero ones)
        out[b] = np.minimum(d, dmax).reshape(D, H, W)
    return out


def input_features(solid, dmax=12.0):
    """Network input [B][D][H][W][16] float64: solid and fluid indicators,
    d/dmax and (d/dmax)^2 with d = chamfer_distance(solid, dmax), zeros."""
    import numpy as np
    solid = np.asarray(solid, dtype=bool)
    q = chamfer_distance(solid, dmax) / dmax
    x = np.zeros(solid.shape + (16,))
    x[..., 0] = solid
    x[..., 1] = ~solid
    x[..., 2] = q
    x[..., 3] = q * q
    return torch.from_numpy(x)
