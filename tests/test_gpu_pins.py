"""Element-wise pins of the solver's set-up and verification calls:
lbm_init_fields against the oracle's equilibrium in every form, and
lbm_verify(LBM_VERIFY_DUCT) against the oracle's duct series on a converged
duct (the verification flow of the paper, Sect. 2.1)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1711_11468_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_11468_amd import lbm
    lbm.load()
    return lbm


INIT_FORMS = [
    {"bounce": "fullway"}, {"bounce": "halfway"},
    {"layout": "aos", "bounce": "fullway"}, {"layout": "aos", "bounce": "halfway"},
    {"addressing": "list", "bounce": "halfway"},
    {"addressing": "list", "bounce": "halfway", "layout": "aos"},
    {"addressing": "ria", "bounce": "halfway"},
    {"propagation": "aa", "bounce": "fullway"}, {"propagation": "aa", "bounce": "halfway"},
    {"propagation": "aa", "layout": "aos", "bounce": "fullway"},
    {"propagation": "aa", "addressing": "list", "bounce": "halfway"},
    {"propagation": "aa", "addressing": "ria", "bounce": "halfway"},
    {"propagation": "push", "bounce": "fullway"}, {"propagation": "push", "bounce": "halfway"},
    {"propagation": "push", "layout": "aos", "bounce": "fullway"},
    {"propagation": "push", "addressing": "list", "bounce": "halfway"},
    {"propagation": "push", "addressing": "ria", "bounce": "halfway"},
]


@pytest.mark.parametrize("kw", INIT_FORMS)
def test_init_fields_is_the_oracle_equilibrium(L, kw):
    """After lbm_init_fields(rho, u) the exported canonical state is, node
    by node, the oracle's equilibrium at (rho, u - g/(2 rho)) on fluid nodes
    (the state then reports velocity u, which includes half the force), and
    the rest state on solid nodes (zeros where half-way solids hold no
    state); within 1e-15 of max |e| (the arithmetic differs only by
    rounding).  A wrong quadratic pair of the equilibrium that keeps rho and
    j exact fails here."""
    import torch
    mask = I.random_solid_mask(16, 12, 10, seed=11, fraction=0.2)
    n = mask.size
    rng = np.random.default_rng(3)
    rho = 1.0 + 1e-2 * rng.uniform(-1, 1, n)
    u = 3e-2 * rng.uniform(-1, 1, (3, n))
    g = np.array([2e-4, -1e-4, 5e-5])
    lat = L.Lattice(mask, g=tuple(g), **kw)
    dev = lat.device
    lat.init_fields(torch.from_numpy(rho).to(dev), torch.from_numpy(u.reshape(-1)).to(dev))
    got = lat.export()
    want = np.zeros((n, 19))
    c, w, _ = O.table()
    solid = mask.reshape(-1) != 0
    for k in range(n):
        if solid[k]:
            want[k] = 0.0 if kw["bounce"] == "halfway" else w
        else:
            want[k] = O.equilibrium(rho[k], u[:, k] - g / (2.0 * rho[k]))
    err = np.abs(got - want).max() / np.abs(want).max()
    assert err <= 1e-15, err
    # a wrong quadratic pair that keeps rho and j exact, 4 (c.u)^2 - 4/3 u^2
    # in place of 9/2 (c.u)^2 - 3/2 u^2, moves the fluid populations by far
    # more than the tolerance at these velocities
    fl = ~solid
    us = (u[:, fl] - g[:, None] / (2.0 * rho[fl])).T
    cu = us @ c.T
    wrong = w * rho[fl, None] * (1 + 3 * cu + 4 * cu ** 2 - (4.0 / 3.0) * (us ** 2).sum(1)[:, None])
    assert np.abs(wrong - want[fl]).max() / np.abs(want).max() > 1e-5


@pytest.fixture(scope="module")
def converged_ducts(L):
    """Rectangular ducts (x periodic, walls on the y and z faces) run to a
    velocity residual below 1e-11: the 4 x 20 x 16 duct and the same duct
    with every width doubled (4 x 38 x 30)."""
    phys = dict(tau_plus=0.8, magic=3 / 16, g=(1e-5, 0.0, 0.0))
    out = {}
    for ny, nz in ((20, 16), (38, 30)):
        mask = I.channel_mask(4, ny, nz)
        # the slowest duct mode decays over ~H^2/(2 pi^2 nu) steps; a
        # stronger force at the wider duct keeps u_max the same
        g = (phys["g"][0] * (16 / (ny - 2)) ** 2, 0.0, 0.0)
        lat = L.Lattice(mask, tau_plus=phys["tau_plus"], magic=phys["magic"], g=g,
                        bounce="halfway")
        steps, r, why = lat.run_to_steady(1e-11, max_steps=400000)
        assert why == "converged", (ny, nz, steps, r)
        out[(ny, nz)] = (lat, mask, g)
    return out


def test_verify_duct_matches_oracle_series(L, converged_ducts):
    """lbm_verify(LBM_VERIFY_DUCT) on a converged rectangular duct returns
    the max-abs and relative L2 error of the velocity against the duct
    series, its max and the compared-node count exactly as the same
    quantities computed on the host from the exported velocity and the
    oracle's series (401 terms, the library's truncation).  The duct is not
    square, so swapped half-widths would show."""
    for (ny, nz), (lat, mask, g) in converged_ducts.items():
        nu = (0.8 - 0.5) / 3.0
        v = lat.verify(L.VERIFY_DUCT)
        u = lat.macroscopic(fields=True)["u"].cpu().numpy().reshape(3, *mask.shape)
        ser = O.duct_series(ny, nz, nu, g[0], terms=401)          # [nz][ny]
        ref = np.zeros_like(u)
        ref[0] = ser[:, :, None]
        fl = mask == 0
        e = (u - ref)[:, fl]
        r = ref[:, fl]
        assert v["n_compared"] == int(fl.sum())
        assert v["ref_max"] == pytest.approx(np.abs(r).max(), rel=1e-12)
        assert v["max_abs"] == pytest.approx(np.abs(e).max(), rel=1e-9)
        assert v["rel_l2"] == pytest.approx(np.sqrt((e ** 2).sum() / (r ** 2).sum()), rel=1e-9)
        # the converged lattice flow is close to the series (a second-order
        # scheme at 14-28 nodes across) and is x-invariant
        assert v["rel_l2"] < 2e-2
        assert np.abs(u - u[:, :, :, :1]).max() <= 1e-15


def test_verify_duct_second_order(L, converged_ducts):
    """Doubling the duct's widths (force scaled to keep u_max) cuts the
    relative L2 error of lbm_verify(LBM_VERIFY_DUCT) by about 4: the
    device's series and the lattice flow converge at second order."""
    e1 = converged_ducts[(20, 16)][0].verify(L.VERIFY_DUCT)["rel_l2"]
    e2 = converged_ducts[(38, 30)][0].verify(L.VERIFY_DUCT)["rel_l2"]
    print("duct rel L2", e1, e2, e1 / e2)
    assert 3.0 < e1 / e2 < 5.5
