"""Seeded synthetic inputs shared by the GPU path and the oracle.

This module holds geometry masks and random numbers only.  It contains none
of the lattice Boltzmann arithmetic, imports nothing from the GPU binding or
from the oracle, and every generator is deterministic given its arguments.

Masks are ``uint8`` arrays of shape ``(nz, ny, nx)`` in C order, so the
linear node index is ``x + nx*(y + ny*z)``; 1 marks a solid node.

Geometries (paper Sect. 2 describes the synthetic domains):
  * ``channel``: empty rectangular duct.  The dimensions include one solid
    wall layer on each y and z face and x is all fluid, so a
    500x100x100 channel has 500*98*98 = 4,802,000 fluid nodes (the count the
    paper quotes in Sect. 4.4).
  * ``slab``: fluid between two plates normal to z, periodic in x and y
    (the verification set-up of Sect. 2.1).
  * ``pipe``: staircase circular cross-section along x (Sect. 2).
  * ``blocks``: equidistant cubic obstacles (Sect. 2).
  * ``spheres``: random spheres placed from a SplitMix64 stream until a
    target voxel porosity is reached (porous-media workload for the list
    representation, Sect. 3 "Lattice Representation").
"""
from __future__ import annotations

import numpy as np

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), a counter-based
    64-bit generator: state advances by the golden-ratio increment and each
    output is the state passed through a fixed xor-shift-multiply mixer."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def channel_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    """Duct along x: solid iff y in {0, ny-1} or z in {0, nz-1}."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[:, 0, :] = 1
    m[:, ny - 1, :] = 1
    m[0, :, :] = 1
    m[nz - 1, :, :] = 1
    return m


def slab_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    """Two plates normal to z (z = 0 and z = nz-1); x and y open."""
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    m[0, :, :] = 1
    m[nz - 1, :, :] = 1
    return m


def pipe_mask(nx: int, ny: int, nz: int) -> np.ndarray:
    """Staircase circular pipe along x inscribed in the y-z cross-section:
    a node is fluid iff its centre lies strictly inside the circle of
    diameter min(ny, nz) - 2 centred in the cross-section."""
    yc = (ny - 1) / 2.0
    zc = (nz - 1) / 2.0
    r = (min(ny, nz) - 2) / 2.0
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[:, None, None]
    inside = (y - yc) ** 2 + (z - zc) ** 2 < r * r
    m = np.where(inside, 0, 1).astype(np.uint8)
    return np.broadcast_to(m, (nz, ny, nx)).copy()


def blocks_mask(nx: int, ny: int, nz: int, block: int, gap: int) -> np.ndarray:
    """Channel with equidistant cubic obstacles of edge ``block`` separated
    by ``gap`` fluid nodes in every direction, inside the duct walls."""
    m = channel_mask(nx, ny, nz)
    period = block + gap
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None] - 1
    z = np.arange(nz)[:, None, None] - 1
    inb = ((x % period) >= gap) & ((y % period) >= gap) & ((z % period) >= gap)
    m[inb & (y >= 0) & (z >= 0)] = 1
    return m


def spheres_mask(nx: int, ny: int, nz: int, seed: int, porosity: float,
                 rmin: float, rmax: float, overlap: bool = True,
                 max_rejects: int = 20000):
    """Random spheres on a fully periodic box.

    Centres are uniform in the box and radii uniform in [rmin, rmax], drawn
    from SplitMix64(seed) in the order (cx, cy, cz, r).  A voxel is solid iff
    the minimum-image distance from its centre (integer coordinates) to a
    sphere centre is <= r.  With ``overlap=True`` spheres are added until the
    voxel porosity is <= ``porosity``.  With ``overlap=False`` a sphere that
    would intersect an earlier one is rejected and placement stops at the
    target or after ``max_rejects`` consecutive rejections (jamming).

    Returns ``(mask, achieved_porosity, n_spheres)``.
    """
    rng = SplitMix64(seed)
    m = np.zeros((nz, ny, nx), dtype=np.uint8)
    n_total = nx * ny * nz
    n_solid = 0
    dims = np.array([nx, ny, nz], dtype=np.float64)
    centres = []
    radii = []
    rejects = 0
    while n_solid < (1.0 - porosity) * n_total:
        c = np.array([rng.uniform() * nx, rng.uniform() * ny, rng.uniform() * nz])
        r = rmin + rng.uniform() * (rmax - rmin)
        if not overlap and centres:
            d = np.array(centres) - c
            d -= dims * np.round(d / dims)
            if np.any(np.sqrt((d * d).sum(axis=1)) < np.array(radii) + r):
                rejects += 1
                if rejects >= max_rejects:
                    break
                continue
        rejects = 0
        centres.append(c)
        radii.append(r)
        ri = int(np.ceil(r)) + 1
        xs = np.arange(int(np.floor(c[0])) - ri, int(np.floor(c[0])) + ri + 2)
        ys = np.arange(int(np.floor(c[1])) - ri, int(np.floor(c[1])) + ri + 2)
        zs = np.arange(int(np.floor(c[2])) - ri, int(np.floor(c[2])) + ri + 2)
        dx = _min_image(xs - c[0], nx)
        dy = _min_image(ys - c[1], ny)
        dz = _min_image(zs - c[2], nz)
        inside = (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 +
                  dx[None, None, :] ** 2) <= r * r
        zi = np.mod(zs, nz)[:, None, None]
        yi = np.mod(ys, ny)[None, :, None]
        xi = np.mod(xs, nx)[None, None, :]
        zi, yi, xi = np.broadcast_arrays(zi, yi, xi)
        sel = inside
        # a box wider than the domain can list a voxel twice; unique() fixes it
        lin = np.unique((xi[sel] + nx * (yi[sel] + ny * zi[sel])).ravel())
        flat = m.reshape(-1)
        new = lin[flat[lin] == 0]
        flat[new] = 1
        n_solid += int(new.size)
    achieved = 1.0 - n_solid / n_total
    return m, achieved, len(centres)


def _min_image(d: np.ndarray, n: int) -> np.ndarray:
    return d - n * np.round(d / n)


def uniform_pm1(shape, seed: int) -> np.ndarray:
    """Seeded uniform numbers in [-1, 1) (PCG64 via numpy), float64."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=shape)


def random_solid_mask(nx: int, ny: int, nz: int, seed: int,
                      fraction: float) -> np.ndarray:
    """Each node solid with probability ``fraction`` (seeded, i.i.d.)."""
    r = np.random.default_rng(seed).random((nz, ny, nx))
    return (r < fraction).astype(np.uint8)
