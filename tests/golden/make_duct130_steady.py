"""Writes two oracle fixtures of the 130 x 130 duct (walls on the y and z
faces, x periodic, half-way bounce-back, tau+ = 0.8, Lambda = 3/16,
g_x = 1e-6, started at rest):

  duct130_step20000.txt  u after exactly 20,000 updates;
  duct130_steady.txt     u once the velocity residual over 500 updates
                         has fallen below 1e-10 (steady state).

Calls only the oracle (its OpenMP build, whose results equal the serial
build's).  The flow does not depend on x, so the oracle runs on a
one-node-thick section.  Each file stores two blocks, u_x then u_y, each on
the quadrant y, z = 0..64 (solid layer included) row by row (z outer).  The
rest follows from the symmetries of the square duct: the mirrors
y -> 129 - y and z -> 129 - z (u_x even in both; u_y odd in y, even in z)
and the swap y <-> z, which exchanges u_y and u_z.  While the flow is still
developing it carries small transverse components (|u_y| ~ 3e-8 at 20,000
updates), so they are stored too.

    python tests/golden/make_duct130_steady.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_1711_11468_amd import inputs as I  # noqa: E402

N = 130
TAU, MAGIC, G = 0.8, 3.0 / 16.0, (1e-6, 0.0, 0.0)
TOL = 1e-10
FIXED = 20000


def _write(name, u, note):
    ux = u[:, 0].reshape(N, N)
    uy = u[:, 1].reshape(N, N)
    uz = u[:, 2].reshape(N, N)
    asym = max(np.abs(ux - ux[::-1, :]).max(), np.abs(ux - ux[:, ::-1]).max(),
               np.abs(ux - ux.T).max(), np.abs(uy + uy[:, ::-1]).max(),
               np.abs(uy - uy[::-1, :]).max(), np.abs(uz - uy.T).max())
    half = N // 2
    path = os.path.join(HERE, name)
    with open(path, "w") as fh:
        fh.write("# oracle u_x then u_y, duct 130x130 cross-section, half-way bounce-back, "
                 "tau+=0.8 Lambda=3/16 g_x=1e-6, rest start\n")
        fh.write("# %s; max-asymmetry %.3e; max |u_y| %.3e; quadrant y,z = 0..%d, z outer\n"
                 % (note, asym, np.abs(uy).max(), half - 1))
        for comp in (ux, uy):
            for z in range(half):
                fh.write(" ".join("%.17g" % v for v in comp[z, :half]) + "\n")
    print("wrote", path, note, flush=True)


def main():
    mask = I.channel_mask(1, N, N)
    t0 = time.time()
    f = O.run(mask, O.rest_state(mask, 1), FIXED, TAU, MAGIC, G, 1, omp=True)
    _write("duct130_step20000.txt", O.macroscopic(mask, f, G)[1],
           "after %d updates" % FIXED)
    f, steps, r = O.run_to_steady(mask, f, TAU, MAGIC, G, 1, TOL, check_every=500, omp=True)
    _write("duct130_steady.txt", O.macroscopic(mask, f, G)[1],
           "steady: %d updates, residual over 500 updates %.3e" % (FIXED + steps, r))
    print("%.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
