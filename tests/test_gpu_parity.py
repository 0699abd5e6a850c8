"""GPU parity: the HIP sweeps against the CPU oracle, element by element.

All comparisons use the canonical pre-collision populations exported by the
library.  FP64 paths must agree with the oracle within 1e-12 relative
max-abs (max |f_gpu - f_oracle| / max |f_oracle|).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1711_11468_amd import inputs as I
from tests._util import BOUNCE, oracle_window_sample, random_state, rel_maxabs

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_11468_amd import lbm
    lbm.load()
    return lbm


def _case(mask, steps, L, f0=None, **kw):
    phys = dict(tau_plus=kw.pop("tau_plus", 0.8), magic=kw.pop("magic", 3 / 16),
                g=kw.pop("g", (1e-6, 0.0, 0.0)))
    bounce = kw.get("bounce", "fullway")
    lat = L.Lattice(mask, **phys, **kw)
    if f0 is not None:
        lat.import_(f0)
    lat.step(steps)
    got = lat.export()
    start = f0 if f0 is not None else O.rest_state(mask, BOUNCE[bounce])
    ref = O.run(mask, start, steps, phys["tau_plus"], phys["magic"], phys["g"], BOUNCE[bounce])
    return got, ref, lat


def test_channel_64x32x32_200_steps_soa(L):
    """Plain D3Q19 TRT fp64 on the 64x32x32 channel (x periodic, full-way
    walls), g_x = 1e-6, tau+ = 0.8, Lambda = 3/16, rest start, 200 steps."""
    mask = I.channel_mask(64, 32, 32)
    got, ref, lat = _case(mask, 200, L)
    print("parity rel max-abs", rel_maxabs(got, ref))
    assert rel_maxabs(got, ref) <= TOL
    _, w, _ = O.table()
    h_err = np.abs(got - ref).max() / np.abs(ref - w).max()
    assert h_err <= 1e-9  # the flow part of the populations (f - w) agrees too
    assert np.abs(ref - w).max() > 1e-6  # the flow has actually developed


@pytest.mark.parametrize("layout,bounce", [("soa", "fullway"), ("soa", "halfway"),
                                           ("aos", "fullway"), ("aos", "halfway")])
@pytest.mark.parametrize("shape", [(9, 10, 12), (5, 7, 131), (100, 21, 45)])
def test_direct_random_state(L, layout, bounce, shape):
    """Random solids (~20 %), random populations and a 3-component force:
    any index or sign error shows.  (5, 7, 131): rows longer than one
    workgroup pass with a ragged tail.  (100, 21, 45): the AoS sweep's
    32 x 8 columns end ragged in x and y and march four z chunks."""
    nz, ny, nx = shape
    mask = I.random_solid_mask(nx, ny, nz, seed=3, fraction=0.2)
    f0 = random_state(mask, seed=9, amplitude=0.02, bounce=bounce)
    got, ref, _ = _case(mask, 25, L, f0=f0, layout=layout, bounce=bounce, block=64,
                        g=(1e-4, -2e-5, 3e-5), tau_plus=0.7, magic=1 / 4)
    assert rel_maxabs(got, ref) <= TOL


@pytest.mark.parametrize("layout", ["soa", "aos"])
@pytest.mark.parametrize("shape", [(9, 10, 12), (6, 9, 70)])
def test_list_random_state(L, shape, layout):
    nz, ny, nx = shape
    mask = I.random_solid_mask(nx, ny, nz, seed=5, fraction=0.3)
    f0 = random_state(mask, seed=4, amplitude=0.02, bounce="halfway")
    got, ref, lat = _case(mask, 25, L, f0=f0, addressing="list", bounce="halfway", layout=layout,
                          g=(-3e-5, 1e-4, 2e-5), tau_plus=1.1, magic=1 / 12)
    assert lat.n_fluid == int((mask == 0).sum())
    assert rel_maxabs(got, ref) <= TOL


def test_pipe_all_addressings(L):
    """Staircase circular pipe (the pipe geometry of Sect. 2) for every
    addressing, both bounce-back kinds on the full array."""
    mask = I.pipe_mask(37, 18, 17)
    for kw in ({"addressing": "list", "bounce": "halfway"}, {"addressing": "ria", "bounce": "halfway"},
               {"addressing": "direct", "bounce": "halfway"}, {"addressing": "direct", "bounce": "fullway"},
               {"layout": "aos", "bounce": "fullway"},
               {"layout": "aos", "addressing": "list", "bounce": "halfway"}):
        got, ref, _ = _case(mask, 30, L, g=(1e-5, 0.0, 0.0), **kw)
        assert rel_maxabs(got, ref) <= TOL, kw


def test_spheres_list_and_direct(L):
    """Porous box of overlapping spheres, fully periodic, both addressings."""
    mask, phi, _ = I.spheres_mask(40, 36, 32, seed=1, porosity=0.5, rmin=3, rmax=6)
    for kw in ({"addressing": "list", "bounce": "halfway"},
               {"addressing": "direct", "bounce": "halfway"},
               {"addressing": "direct", "bounce": "fullway"}):
        got, ref, _ = _case(mask, 40, L, **kw)
        assert rel_maxabs(got, ref) <= TOL, kw


def test_import_export_roundtrip(L):
    """Import followed by export returns the canonical state bit for bit."""
    mask = I.random_solid_mask(11, 7, 6, seed=8, fraction=0.25)
    for kw in ({"layout": "soa", "bounce": "fullway"}, {"layout": "aos", "bounce": "halfway"},
               {"addressing": "list", "bounce": "halfway"}, {"addressing": "ria", "bounce": "halfway"},
               {"addressing": "ria", "bounce": "halfway", "propagation": "aa"},
               {"addressing": "list", "bounce": "halfway", "layout": "aos"}):
        f0 = random_state(mask, seed=1, amplitude=0.05, bounce=kw["bounce"])
        lat = L.Lattice(mask, **kw)
        lat.import_(f0)
        assert np.array_equal(lat.export(), f0), kw


def test_block_size_bitwise_and_layouts_agree(L):
    """Results do not depend on the workgroup size (bitwise: no races, no
    order dependence) and SoA, AoS and list (all half-way) agree to
    round-off (the compiler may contract multiply-adds differently)."""
    mask = I.random_solid_mask(150, 6, 5, seed=2, fraction=0.15)
    f0 = random_state(mask, seed=3, amplitude=0.02, bounce="halfway")

    def run(**kw):
        lat = L.Lattice(mask, bounce="halfway", g=(1e-5, 0, 0), **kw)
        lat.import_(f0)
        lat.step(12)
        return lat.export()

    for base, blocks in (({}, (64, 128, 256, 1024)), ({"layout": "aos"}, (64, 256, 512)),
                         ({"addressing": "list"}, (64, 256, 1024)),
                         ({"addressing": "list", "layout": "aos"}, (64, 256, 512))):
        outs = [run(block=b, **base) for b in blocks]
        for o in outs[1:]:
            assert np.array_equal(o, outs[0]), base
    ref = run()
    for kw in ({"layout": "aos"}, {"addressing": "list"}, {"addressing": "list", "layout": "aos"}):
        assert rel_maxabs(run(**kw), ref) <= 1e-15, kw


@pytest.mark.parametrize("layout,prop", [("soa", "os"), ("aos", "os"), ("soa", "push"),
                                         ("aos", "push"), ("soa", "aa"), ("aos", "aa")])
def test_full_size_channel_512_sampled(L, layout, prop):
    """512^3 channel in the benchmark's launch configuration (every 512^3
    form the benchmark times): sampled nodes (corners, walls, interior)
    against the windowed oracle after 12 steps, and every x-slice identical
    (x-invariance of the duct flow)."""
    n, steps = 512, 12
    mask = I.channel_mask(n, n, n)
    phys = dict(tau_plus=0.8, magic=3 / 16, g=(1e-6, 0.0, 0.0))
    lat = L.Lattice(mask, layout=layout, propagation=prop, **phys)
    lat.step(steps)
    pts = [(0, 1, 1), (5, 1, 2), (511, 2, 1), (100, 255, 256), (7, 510, 510), (300, 1, 300),
           (0, 0, 0), (400, 511, 17)]
    ids = [x + n * (y + n * z) for x, y, z in pts]
    got = lat.export(ids)
    for k, c in enumerate(pts):
        ref = oracle_window_sample(mask, c, steps, **phys)
        assert rel_maxabs(got[k], ref) <= TOL, c
    # x-invariance on one cross-section line
    row = [x + n * (3 + n * 2) for x in range(0, n, 37)]
    vals = lat.export(row)
    assert np.array_equal(vals, np.repeat(vals[:1], len(row), axis=0))
    st = lat.macroscopic()
    # mass over all nodes (walls hold populations in transit) is conserved
    assert abs(st["mass"] - n ** 3) <= 1e-12 * n ** 3
    if prop == "os":
        # the fused sweep + diagnostics on the same state: the same stats
        # (its records exceed one reduction stage) and a zero residual
        sd = lat.step_diag()
        assert sd["step"] == st["step"] and sd["residual"] == 0.0
        assert abs(sd["mass"] - st["mass"]) <= 1e-13 * st["mass"]
        assert sd["u_max"] == st["u_max"]
        np.testing.assert_allclose(sd["momentum"], st["momentum"], rtol=1e-12, atol=1e-9)


@pytest.fixture(scope="module")
def spheres384():
    return I.spheres_mask(384, 384, 384, seed=0, porosity=0.4, rmin=8, rmax=16)[0]


@pytest.mark.parametrize("addressing,layout,prop", [
    ("list", "soa", "os"), ("list", "soa", "aa"), ("list", "soa", "push"),
    ("ria", "soa", "os"), ("ria", "soa", "aa"),
    ("list", "aos", "os"), ("list", "aos", "aa"), ("list", "aos", "push"),
    ("direct", "soa", "os")])
def test_full_size_spheres_384_list_sampled(L, spheres384, addressing, layout, prop):
    """384^3 porous box in every form the benchmark times on it (fluid list
    plain or run-length, SoA or AoS records, pull, AA, push; the full array
    with link words) against the windowed oracle."""
    n, steps = 384, 8
    mask = spheres384
    phys = dict(tau_plus=0.8, magic=3 / 16, g=(1e-6, 0.0, 0.0))
    lat = L.Lattice(mask, addressing=addressing, layout=layout, propagation=prop,
                    bounce="halfway", **phys)
    lat.step(steps)
    rng = np.random.default_rng(7)
    fluid = np.flatnonzero(mask.reshape(-1) == 0)
    ids = rng.choice(fluid, 12, replace=False)
    got = lat.export(ids)
    for k, lin in enumerate(ids):
        c = (int(lin % n), int((lin // n) % n), int(lin // (n * n)))
        ref = oracle_window_sample(mask, c, steps, bounce="halfway", **phys)
        assert rel_maxabs(got[k], ref) <= TOL, c


def test_diagnostics_mass_momentum(L):
    """Mass is conserved and momentum grows by Nf g per step (no solids)."""
    mask = np.zeros((6, 7, 9), dtype=np.uint8)
    g = np.array([1e-4, -2e-5, 5e-5])
    f0 = random_state(mask, seed=6, amplitude=0.02, bounce="fullway")
    lat = L.Lattice(mask, g=tuple(g))
    lat.import_(f0)
    s0 = lat.macroscopic()
    lat.step(7)
    s1 = lat.macroscopic()
    assert abs(s1["mass"] - s0["mass"]) <= 1e-13 * s0["mass"]
    np.testing.assert_allclose(np.array(s1["momentum"]) - np.array(s0["momentum"]),
                               7 * mask.size * g, atol=1e-13)
    # fields agree with the oracle's macroscopic quantities
    ref = O.run(mask, f0, 7, 0.8, 3 / 16, g, 0)
    rho_o, u_o = O.macroscopic(mask, ref, g)
    s2 = lat.macroscopic(fields=True)
    np.testing.assert_allclose(s2["rho"].cpu().numpy(), rho_o, rtol=1e-13)
    np.testing.assert_allclose(s2["u"].cpu().numpy().T, u_o, atol=1e-15)


def test_residual_and_slab_verify(L):
    """Run the slab to steady state with the residual driver and verify the
    parabola (Lambda = 3/16 makes it exact)."""
    mask = I.slab_mask(4, 4, 12)
    lat = L.Lattice(mask, g=(1e-5, 0, 0), bounce="halfway")
    lat.macroscopic()
    r = 1.0
    for _ in range(200):
        lat.step(100)
        r = lat.macroscopic()["residual"]
        if r < 1e-12:
            break
    assert r < 1e-12
    v = lat.verify(L.VERIFY_SLAB)
    assert v["rel_l2"] < 1e-10
    assert v["n_compared"] == 4 * 4 * 10


def test_nonfinite_detected(L):
    mask = I.channel_mask(8, 6, 6)
    lat = L.Lattice(mask)
    f = O.rest_state(mask, 0)
    f[2 + 8 * (2 + 6 * 2), 3] = np.nan
    lat.import_(f)
    st = lat.macroscopic(allow_nonfinite=True)
    assert st["rc"] == L.ENONFINITE and st["nonfinite"] >= 1


_DIAG_FORMS = [
    {"bounce": "fullway"}, {"bounce": "halfway"},
    {"bounce": "fullway", "storage": "f32s"}, {"bounce": "halfway", "storage": "f16sr"},
    # the AoS column march carries them too
    {"layout": "aos", "bounce": "halfway"}, {"layout": "aos", "bounce": "fullway", "storage": "f32s"},
    # forms without a fused sweep run the two passes in turn
    {"addressing": "list", "bounce": "halfway"},
    {"propagation": "aa", "bounce": "fullway"}, {"propagation": "push", "bounce": "halfway"},
]


@pytest.mark.parametrize("kw", _DIAG_FORMS)
@pytest.mark.parametrize("shape", [(70, 9, 11), (5, 72, 64)])
def test_step_diag_matches_separate_passes(L, kw, shape):
    """lbm_step_diag = lbm_macroscopic then lbm_step(1): the same stats
    (sums to FP64 rounding of a different fixed order; max |u| and the count
    exactly) and the same state; the rows of (5, 72, 64) exceed one
    reduction stage.  FP64 states also match the oracle."""
    mask = I.random_solid_mask(*shape, seed=21, fraction=0.15)
    bounce = kw["bounce"]
    f0 = random_state(mask, seed=8, amplitude=0.02, bounce=bounce)
    phys = dict(tau_plus=0.7, magic=3 / 16, g=(2e-5, -1e-5, 3e-6))
    fused = L.Lattice(mask, **phys, **kw)
    plain = L.Lattice(mask, **phys, **kw)
    fused.import_(f0)
    plain.import_(f0)
    steps = 5
    for k in range(steps):
        a = fused.step_diag()
        b = plain.macroscopic()
        plain.step(1)
        assert a["step"] == b["step"] == k
        assert abs(a["mass"] - b["mass"]) <= 1e-13 * abs(b["mass"])
        np.testing.assert_allclose(a["momentum"], b["momentum"], rtol=0, atol=1e-14 * b["mass"])
        assert a["u_max"] == pytest.approx(b["u_max"], rel=1e-15, abs=0)
        assert a["nonfinite"] == b["nonfinite"] == 0
        if k == 0:
            assert a["residual"] == b["residual"] == -1.0
        else:
            assert b["residual"] > 0
            assert a["residual"] == pytest.approx(b["residual"], rel=1e-12)
    assert fused.step_count == plain.step_count == steps
    got, want = fused.export(), plain.export()
    assert rel_maxabs(got, want) <= 1e-15
    # both histories now hold the velocity of step steps - 1: one more pair
    a = fused.step_diag()
    b = plain.macroscopic()
    assert a["residual"] == pytest.approx(b["residual"], rel=1e-12)
    if kw.get("storage", "f64") == "f64":
        ref = O.run(mask, f0, steps, phys["tau_plus"], phys["magic"], phys["g"], BOUNCE[bounce])
        assert rel_maxabs(got, ref) <= TOL


def test_step_diag_nonfinite(L):
    """A non-finite population in the state the fused sweep reads is
    counted and reported; the update has still run."""
    mask = I.channel_mask(8, 6, 6)
    lat = L.Lattice(mask)
    f = O.rest_state(mask, 0)
    f[2 + 8 * (2 + 6 * 2), 3] = np.nan
    lat.import_(f)
    st = lat.step_diag(allow_nonfinite=True)
    assert st["rc"] == L.ENONFINITE and st["nonfinite"] == 1 and st["step"] == 0
    assert lat.step_count == 1


@pytest.mark.parametrize("kw", [{"addressing": "list", "bounce": "halfway"},
                                {"layout": "aos", "bounce": "fullway"},
                                {"storage": "f32s"}])
def test_init_fields_reports_given_state(L, kw):
    """After lbm_init_fields(rho, u) the diagnostics report exactly that
    density and velocity on fluid nodes (the equilibrium is taken at
    u - g/(2 rho) because the velocity includes half the force)."""
    import torch
    mask = I.random_solid_mask(16, 12, 10, seed=11, fraction=0.2)
    n = mask.size
    rng = np.random.default_rng(3)
    rho = 1.0 + 1e-3 * rng.uniform(-1, 1, n)
    u = 1e-3 * rng.uniform(-1, 1, (3, n))
    lat = L.Lattice(mask, g=(2e-4, -1e-4, 5e-5), **kw)
    dev = lat.device
    lat.init_fields(torch.from_numpy(rho).to(dev), torch.from_numpy(u.reshape(-1)).to(dev))
    st = lat.macroscopic(fields=True)
    fl = mask.reshape(-1) == 0
    tol = 1e-15 if kw.get("storage", "f64") == "f64" else 1e-9
    np.testing.assert_allclose(st["rho"].cpu().numpy()[fl], rho[fl], rtol=0, atol=tol * 1e2)
    np.testing.assert_allclose(st["u"].cpu().numpy()[:, fl], u[:, fl], rtol=0, atol=tol)


@pytest.mark.parametrize("kw", [{"bounce": "fullway"}, {"bounce": "halfway"},
                                {"addressing": "list", "bounce": "halfway"},
                                {"bounce": "fullway", "storage": "f64", "block": 64},
                                {"layout": "aos", "bounce": "fullway"},
                                {"layout": "aos", "bounce": "halfway"},
                                {"layout": "aos", "addressing": "list", "bounce": "halfway"}])
@pytest.mark.parametrize("steps", [24, 25])
def test_aa_pattern_random_state(L, kw, steps):
    """AA pattern (one lattice, alternating local and neighbour kernels)
    against the oracle after an even and an odd number of updates, from a
    random state with random solids and a 3-component force."""
    mask = I.random_solid_mask(70, 9, 7, seed=12, fraction=0.2)
    f0 = random_state(mask, seed=13, amplitude=0.02, bounce=kw["bounce"])
    got, ref, lat = _case(mask, steps, L, f0=f0, propagation="aa", g=(1e-4, 3e-5, -2e-5),
                          tau_plus=0.9, magic=3 / 16, **kw)
    assert rel_maxabs(got, ref) <= TOL
    # mass over the state-holding nodes is conserved
    st = lat.macroscopic()
    assert abs(st["mass"] - f0.sum()) <= 1e-13 * f0.sum()


def test_aa_matches_two_lattice_bitwise_free(L):
    """AA and one-step propagation give the same states (to round-off) on
    the channel, step by step; AA uses one buffer."""
    mask = I.channel_mask(64, 20, 18)
    a = L.Lattice(mask, g=(1e-5, 0, 0), propagation="aa")
    b = L.Lattice(mask, g=(1e-5, 0, 0))
    assert "pdf_b" not in a._t
    for k in range(3):
        a.step(7)
        b.step(7)
        assert rel_maxabs(a.export(), b.export()) <= 1e-15


@pytest.mark.parametrize("kw", [{"bounce": "fullway"}, {"bounce": "halfway"},
                                {"addressing": "list", "bounce": "halfway"},
                                {"bounce": "fullway", "storage": "f64", "block": 64},
                                {"layout": "aos", "bounce": "fullway"},
                                {"layout": "aos", "bounce": "halfway"},
                                {"layout": "aos", "addressing": "list", "bounce": "halfway"}])
def test_push_random_state(L, kw):
    """One-step push kernels (read the node, collide, scatter to the
    neighbours) against the oracle from a random state with random solids
    and a 3-component force, on a row that spans several blocks with a
    ragged tail."""
    mask = I.random_solid_mask(131, 9, 7, seed=14, fraction=0.2)
    f0 = random_state(mask, seed=15, amplitude=0.02, bounce=kw["bounce"])
    got, ref, lat = _case(mask, 13, L, f0=f0, propagation="push", g=(1e-4, 3e-5, -2e-5),
                          tau_plus=0.9, magic=3 / 16, **kw)
    assert rel_maxabs(got, ref) <= TOL
    st = lat.macroscopic()
    assert abs(st["mass"] - f0.sum()) <= 1e-13 * f0.sum()


@pytest.mark.parametrize("prop,steps", [("push", 9), ("aa", 9), ("aa", 10)])
@pytest.mark.parametrize("bounce", ["fullway", "halfway"])
def test_aos_columns_ragged_chunks(L, prop, steps, bounce):
    """The AoS push and AA neighbour step march 32 x 8 columns through z
    chunks: a lattice whose columns end ragged in x and y and whose 100
    layers split into four chunks, against the oracle."""
    mask = I.random_solid_mask(45, 21, 100, seed=16, fraction=0.2)
    f0 = random_state(mask, seed=17, amplitude=0.02, bounce=bounce)
    got, ref, _ = _case(mask, steps, L, f0=f0, propagation=prop, layout="aos", bounce=bounce,
                        g=(1e-4, 3e-5, -2e-5), tau_plus=0.9)
    assert rel_maxabs(got, ref) <= TOL


def test_push_and_pull_agree_stepwise(L):
    """Push and pull one-step sweeps give the same states step by step (to
    round-off) on the channel, and a state imported into a push lattice
    continues like the pull lattice it came from."""
    mask = I.channel_mask(64, 20, 18)
    a = L.Lattice(mask, g=(1e-5, 0, 0), propagation="push")
    b = L.Lattice(mask, g=(1e-5, 0, 0))
    for k in range(3):
        a.step(5)
        b.step(5)
        assert rel_maxabs(a.export(), b.export()) <= 1e-15
    c = L.Lattice(mask, g=(1e-5, 0, 0), propagation="push")
    c.import_(b.export())
    b.step(4)
    c.step(4)
    assert rel_maxabs(c.export(), b.export()) <= 1e-15


@pytest.mark.parametrize("kw", [{}, {"layout": "aos"}, {"bounce": "halfway"}, {"propagation": "aa"},
                                {"propagation": "push"}, {"propagation": "push", "bounce": "halfway"},
                                {"propagation": "aa", "layout": "aos"}, {"propagation": "push", "layout": "aos"},
                                {"addressing": "list", "bounce": "halfway"},
                                {"addressing": "list", "bounce": "halfway", "propagation": "push"},
                                {"addressing": "ria", "bounce": "halfway"},
                                {"addressing": "ria", "bounce": "halfway", "propagation": "aa"},
                                {"addressing": "list", "bounce": "halfway", "layout": "aos"},
                                {"addressing": "list", "bounce": "halfway", "layout": "aos", "propagation": "aa"}])
def test_degenerate_lattices(L, kw):
    """1-node and thin lattices (every neighbour is the node itself or a
    wrap-around), and a geometry without fluid, behave like the oracle."""
    for shape in ((1, 1, 1), (1, 3, 1), (2, 1, 5)):
        mask = np.zeros(shape, dtype=np.uint8)
        bounce = kw.get("bounce", "fullway")
        f0 = random_state(mask, seed=1, amplitude=0.05, bounce=bounce)
        got, ref, _ = _case(mask, 9, L, f0=f0, g=(1e-4, -1e-4, 2e-5), **kw)
        assert rel_maxabs(got, ref) <= TOL, (shape, kw)
    solid = np.ones((3, 4, 5), dtype=np.uint8)
    lat = L.Lattice(solid, **kw)
    lat.step(3)
    st = lat.macroscopic()
    assert st["nonfinite"] == 0 and st["u_max"] == 0.0


def _ria_geometries():
    # short runs (random solids), long runs crossing 64-node chunks (a duct
    # 131 long), and pores of a sphere pack
    duct = I.channel_mask(131, 7, 6)
    spheres, _, _ = I.spheres_mask(70, 12, 10, seed=4, porosity=0.7, rmin=2, rmax=4)
    return {"random": I.random_solid_mask(67, 9, 7, seed=21, fraction=0.3),
            "duct": duct, "spheres": spheres}


@pytest.mark.parametrize("geom", ["random", "duct", "spheres"])
@pytest.mark.parametrize("prop,steps", [("os", 17), ("aa", 24), ("aa", 25), ("push", 17)])
def test_ria_random_state(L, geom, prop, steps):
    """Run-length list (reduced indirect addressing) for every propagation
    form against the oracle, from a random state with a 3-component force."""
    mask = _ria_geometries()[geom]
    f0 = random_state(mask, seed=22, amplitude=0.02, bounce="halfway")
    got, ref, lat = _case(mask, steps, L, f0=f0, addressing="ria", bounce="halfway",
                          propagation=prop, g=(1e-4, -3e-5, 2e-5), tau_plus=0.9, magic=3 / 16)
    assert lat.sizes.n_runs > 0 and lat.sizes.adj_bytes == 0
    assert rel_maxabs(got, ref) <= TOL
    st = lat.macroscopic()
    assert abs(st["mass"] - f0.sum()) <= 1e-13 * f0.sum()


def test_ria_and_list_agree(L):
    """The run-length list reads exactly the slots the adjacency list names:
    both lists give the same states to round-off, step by step, for pull,
    push and AA."""
    mask = _ria_geometries()["spheres"]
    f0 = random_state(mask, seed=5, amplitude=0.02, bounce="halfway")
    for prop in ("os", "push", "aa"):
        a = L.Lattice(mask, addressing="ria", bounce="halfway", propagation=prop, g=(1e-5, 0, 0))
        b = L.Lattice(mask, addressing="list", bounce="halfway", propagation=prop, g=(1e-5, 0, 0))
        a.import_(f0)
        b.import_(f0)
        for _ in range(3):
            a.step(5)
            b.step(5)
            assert rel_maxabs(a.export(), b.export()) <= 1e-15, prop


# the forms the kernel study times on the `blocks` geometry (and the AoS
# forms it times on the channel)
STUDY_FORMS = [
    {}, {"bounce": "halfway"}, {"propagation": "push"},
    {"addressing": "list", "bounce": "halfway"},
    {"addressing": "list", "bounce": "halfway", "propagation": "push"},
    {"addressing": "ria", "bounce": "halfway"},
    {"propagation": "aa"},
    {"addressing": "list", "bounce": "halfway", "propagation": "aa"},
    {"addressing": "ria", "bounce": "halfway", "propagation": "aa"},
    {"layout": "aos"}, {"addressing": "list", "bounce": "halfway", "layout": "aos"},
]


@pytest.mark.parametrize("kw", STUDY_FORMS)
@pytest.mark.parametrize("edge", [1, 2, 3])
def test_blocks_geometry_whole_domain(L, kw, edge):
    """The `blocks` geometry (cubic obstacles of edge b, gap b, inside the
    channel walls; the paper's Fig. 4 study) in every form the kernel study
    times: the whole state against the oracle after an odd number of
    updates."""
    mask = I.blocks_mask(61, 14, 13, block=edge, gap=edge)
    assert 0 < int(mask.sum()) < mask.size
    got, ref, _ = _case(mask, 11, L, **kw)
    assert rel_maxabs(got, ref) <= TOL


@pytest.mark.parametrize("kw", STUDY_FORMS[:9])
@pytest.mark.parametrize("edge", [1, 4, 16])
def test_blocks_study_size_sampled(L, kw, edge):
    """The study's own size (500 x 100 x 100, edges 1, 4, 16): fluid nodes
    next to obstacle faces, edges and corners and in the gaps, against the
    windowed oracle after 8 updates."""
    steps = 8
    mask = I.blocks_mask(500, 100, 100, block=edge, gap=edge)
    phys = dict(tau_plus=0.8, magic=3 / 16, g=(1e-6, 0.0, 0.0))
    lat = L.Lattice(mask, **phys, **kw)
    lat.step(steps)
    fluid = mask == 0
    solid = ~fluid
    # fluid nodes with a solid neighbour among the 18 links, off the walls
    near = np.zeros_like(fluid)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if abs(dx) + abs(dy) + abs(dz) in (1, 2):
                    near |= np.roll(solid, (dz, dy, dx), axis=(0, 1, 2))
    near &= fluid
    near[:, :2, :] = near[:, -2:, :] = False
    near[:2, :, :] = near[-2:, :, :] = False
    rng = np.random.default_rng(edge)
    ids = np.concatenate([rng.choice(np.flatnonzero(near.reshape(-1)), 10, replace=False),
                          rng.choice(np.flatnonzero(fluid.reshape(-1)), 4, replace=False)])
    got = lat.export(ids)
    bounce = kw.get("bounce", "fullway")
    for k, lin in enumerate(ids):
        c = (int(lin % 500), int((lin // 500) % 100), int(lin // 50000))
        ref = oracle_window_sample(mask, c, steps, bounce=bounce, **phys)
        assert rel_maxabs(got[k], ref) <= TOL, (c, kw)
