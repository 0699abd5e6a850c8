"""Pure-Python brute-force D3Q19 TRT update for tiny lattices.

TEST INFRASTRUCTURE ONLY.  A second, deliberately naive transcription of
the same model as ``lbm_oracle.c``, used to cross-check it on 4^3-sized
problems.  It uses no table: the velocity set is enumerated as every
c in {-1,0,1}^3 with |c|^2 <= 2, weights follow from |c|^2 (1/3, 1/18,
1/36), the opposite of c is -c, populations are keyed by (node, c) in
dictionaries and the domain is walked with explicit coordinates.

Model readings (paper Sect. 2 and 3.2 name TRT, bounce-back and a constant
body force; the formulas are the textbook ones): TRT relaxation of the
symmetric/antisymmetric halves, second-order equilibrium, split forcing
with u = (sum c f + g/2)/rho, full-way or half-way bounce-back, periodic
wrap on the axes flagged periodic (all by default).  Beyond the faces of
the other axes every node is solid: under half-way bounce-back a population
leaving the box there is reflected at its node; full-way bounce-back needs
solid nodes on those faces and wraps them (only solids exchange there).
"""
from __future__ import annotations

import itertools


def velocities():
    return [c for c in itertools.product((-1, 0, 1), repeat=3)
            if c[0] * c[0] + c[1] * c[1] + c[2] * c[2] <= 2]


def weight(c):
    n2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2]
    return {0: 1.0 / 3.0, 1: 1.0 / 18.0, 2: 1.0 / 36.0}[n2]


def neg(c):
    return (-c[0], -c[1], -c[2])


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


class Brute:
    def __init__(self, nx, ny, nz, is_solid, tau_plus, magic, g, fullway,
                 periodic=(True, True, True)):
        self.n = (nx, ny, nz)
        self.periodic = tuple(bool(a) for a in periodic)
        self.is_solid = is_solid          # callable (x, y, z) -> bool
        self.lp = 1.0 / tau_plus
        self.lm = 1.0 / (0.5 + magic / (tau_plus - 0.5))
        self.g = tuple(g)
        self.fullway = fullway
        self.vel = velocities()

    def nodes(self):
        nx, ny, nz = self.n
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    yield (x, y, z)

    def shift(self, p, c):
        return tuple((p[a] + c[a]) % self.n[a] for a in range(3))

    def beyond_wall(self, p, c):
        return any(not self.periodic[a] and not 0 <= p[a] + c[a] < self.n[a]
                   for a in range(3))

    def moments(self, fn):
        rho = sum(fn[c] for c in self.vel)
        u = tuple((sum(c[a] * fn[c] for c in self.vel) + 0.5 * self.g[a]) / rho
                  for a in range(3))
        return rho, u

    def collide(self, fn):
        rho, u = self.moments(fn)
        uu = dot(u, u)

        def eq(c):
            cu = dot(c, u)
            return weight(c) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu)

        def force(c):
            cu = dot(c, u)
            return weight(c) * sum((3.0 * (c[a] - u[a]) + 9.0 * cu * c[a]) * self.g[a]
                                   for a in range(3))

        out = {}
        for c in self.vel:
            o = neg(c)
            fp, fm = 0.5 * (fn[c] + fn[o]), 0.5 * (fn[c] - fn[o])
            ep, em = 0.5 * (eq(c) + eq(o)), 0.5 * (eq(c) - eq(o))
            Fp, Fm = 0.5 * (force(c) + force(o)), 0.5 * (force(c) - force(o))
            out[c] = (fn[c] - self.lp * (fp - ep) - self.lm * (fm - em)
                      + (1.0 - 0.5 * self.lp) * Fp + (1.0 - 0.5 * self.lm) * Fm)
        return out

    def step(self, f):
        post = {}
        for p in self.nodes():
            if not self.is_solid(*p):
                post[p] = self.collide(f[p])
            elif self.fullway:
                post[p] = {c: f[p][neg(c)] for c in self.vel}
        new = {p: {} for p in self.nodes()
               if self.fullway or not self.is_solid(*p)}
        for p, fp in post.items():
            for c in self.vel:
                q = self.shift(p, c)
                if self.fullway or not (self.beyond_wall(p, c) or self.is_solid(*q)):
                    new[q][c] = fp[c]
                else:
                    new[p][neg(c)] = fp[c]
        return new
