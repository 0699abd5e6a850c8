"""The windowed oracle used for full-size sampled parity equals the oracle
on the whole domain (also when the window is wider than the domain)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1711_11468_amd import inputs as I
from tests._util import BOUNCE, oracle_window_sample, random_state


@pytest.mark.parametrize("bounce", ["fullway", "halfway"])
def test_window_matches_full_domain(bounce):
    mask, _, _ = I.spheres_mask(14, 12, 9, seed=4, porosity=0.6, rmin=1.5, rmax=3)
    phys = dict(tau_plus=0.8, magic=3 / 16, g=(1e-4, 2e-5, -1e-5))
    f0 = random_state(mask, seed=2, amplitude=0.03, bounce=bounce)
    steps = 6
    full = O.run(mask, f0, steps, phys["tau_plus"], phys["magic"], phys["g"], BOUNCE[bounce])
    nz, ny, nx = mask.shape
    for c in [(0, 0, 0), (13, 11, 8), (5, 6, 4), (7, 0, 3)]:
        got = oracle_window_sample(mask, c, steps, f0_full=f0, bounce=bounce, **phys)
        ref = full[c[0] + nx * (c[1] + ny * c[2])]
        assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max()
