"""Writes two oracle fixtures of the 130 x 130 duct (walls on the y and z
faces, x periodic, half-way bounce-back, tau+ = 0.8, Lambda = 3/16,
g_x = 1e-6, started at rest):

  duct130_step20000.txt  u_x after exactly 20,000 updates;
  duct130_steady.txt     u_x once the velocity residual over 500 updates
                         has fallen below 1e-10 (steady state).

Calls only the oracle (its OpenMP build, whose results equal the serial
build's).  The flow does not depend on x, so the oracle runs on a
one-node-thick section.  Each file stores the quadrant y, z = 0..64 (solid
layer included) row by row (z outer); the rest follows from the mirror
symmetries y -> 129 - y and z -> 129 - z of the duct.

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


def _write(name, ux, note):
    asym = max(np.abs(ux - ux[::-1, :]).max(), np.abs(ux - ux[:, ::-1]).max(),
               np.abs(ux - ux.T).max())
    half = N // 2
    path = os.path.join(HERE, name)
    with open(path, "w") as fh:
        fh.write("# oracle u_x, duct 130x130 cross-section, half-way bounce-back, "
                 "tau+=0.8 Lambda=3/16 g_x=1e-6, rest start\n")
        fh.write("# %s; max-asymmetry %.3e; quadrant y,z = 0..%d, z outer\n"
                 % (note, asym, half - 1))
        for z in range(half):
            fh.write(" ".join("%.17g" % v for v in ux[z, :half]) + "\n")
    print("wrote", path, note, flush=True)


def main():
    mask = I.channel_mask(1, N, N)
    t0 = time.time()
    f = O.run(mask, O.rest_state(mask, 1), FIXED, TAU, MAGIC, G, 1, omp=True)
    _write("duct130_step20000.txt", O.macroscopic(mask, f, G)[1][:, 0].reshape(N, N),
           "after %d updates" % FIXED)
    f, steps, r = O.run_to_steady(mask, f, TAU, MAGIC, G, 1, TOL, check_every=500, omp=True)
    _write("duct130_steady.txt", O.macroscopic(mask, f, G)[1][:, 0].reshape(N, N),
           "steady: %d updates, residual over 500 updates %.3e" % (FIXED + steps, r))
    print("%.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
