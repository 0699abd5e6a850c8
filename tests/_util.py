"""Shared test helpers: oracle comparisons and windowed oracle samples."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

BOUNCE = {"fullway": 0, "halfway": 1}


def rel_maxabs(a, b):
    """max |a - b| / max |b| (the parity norm on populations)."""
    return float(np.abs(a - b).max() / np.abs(b).max())


def random_state(mask, seed, amplitude, bounce):
    """w_i (1 + amplitude * U(-1, 1)) per node and direction (oracle weights);
    nodes without state (half-way solids) are zero."""
    _, w, _ = O.table()
    from paper_1711_11468_amd import inputs as I
    eps = I.uniform_pm1((mask.size, 19), seed)
    f = w[None, :] * (1.0 + amplitude * eps)
    if bounce == "halfway":
        f[mask.reshape(-1) != 0] = 0.0
    return f


def window_indices(center, shape, radius):
    """Wrapped index vectors of the (2r+1)^3 window around (x, y, z)."""
    nz, ny, nx = shape
    x0, y0, z0 = center
    r = np.arange(-radius, radius + 1)
    return (np.mod(z0 + r, nz), np.mod(y0 + r, ny), np.mod(x0 + r, nx))


def oracle_window_sample(mask, center, steps, f0_full=None, bounce="fullway", **phys):
    """Oracle populations of node ``center`` after ``steps`` updates, from a
    (2*steps+1)^3 window of the (periodic) domain: a node only depends on
    nodes within L-inf distance ``steps`` and the window's own wrap reaches
    the centre after steps+1 updates, so the result equals the full-domain
    one.  ``f0_full``: initial canonical state [N][19] (default: rest)."""
    zi, yi, xi = window_indices(center, mask.shape, steps)
    wmask = np.ascontiguousarray(mask[np.ix_(zi, yi, xi)])
    b = BOUNCE[bounce]
    if f0_full is None:
        f0 = O.rest_state(wmask, b)
    else:
        nz, ny, nx = mask.shape
        lin = (xi[None, None, :] + nx * (yi[None, :, None] + ny * zi[:, None, None])).reshape(-1)
        f0 = f0_full[lin]
    f = O.run(wmask, f0, steps, phys["tau_plus"], phys["magic"], phys["g"], b)
    c = steps
    w = 2 * steps + 1
    return f[c + w * (c + w * c)]


def golden_duct130(name):
    """Full 130 x 130 cross-section u[3][z][y] of a duct fixture in
    tests/golden/ (stored as u_x and u_y on the quadrant y, z = 0..64; the
    square duct is mirror-symmetric in y and z, u_y odd in y, and the swap
    y <-> z exchanges u_y and u_z)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    q = np.loadtxt(path)
    h = q.shape[1]
    qx, qy = q[:h], q[h:]

    def unfold(quad, ysign):
        top = np.concatenate([quad, ysign * quad[:, ::-1]], axis=1)
        return np.concatenate([top, top[::-1, :]], axis=0)
    ux = unfold(qx, 1.0)
    uy = unfold(qy, -1.0)
    return np.stack([ux, uy, uy.T])
