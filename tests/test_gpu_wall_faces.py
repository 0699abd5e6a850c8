"""GPU parity on boxes with axes that do not wrap (periodicity per axis,
paper Sect. 3.2): the faces of those axes are walls and nodes beyond them
count as solid.  Every addressing, layout and propagation form against the
oracle run with the same periodic bits, element by element."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1711_11468_amd import inputs as I
from tests._util import BOUNCE, random_state, rel_maxabs

pytestmark = pytest.mark.gpu

TOL = 1e-12

FORMS = [
    {}, {"layout": "aos"}, {"propagation": "aa"}, {"propagation": "push"},
    {"layout": "aos", "propagation": "aa"}, {"layout": "aos", "propagation": "push"},
    {"addressing": "list"}, {"addressing": "list", "propagation": "aa"},
    {"addressing": "list", "propagation": "push"}, {"addressing": "list", "layout": "aos"},
    {"addressing": "list", "layout": "aos", "propagation": "aa"},
    {"addressing": "list", "layout": "aos", "propagation": "push"},
    {"addressing": "ria"}, {"addressing": "ria", "propagation": "aa"},
    {"addressing": "ria", "propagation": "push"},
]


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1711_11468_amd import lbm
    lbm.load()
    return lbm


def _run(L, mask, f0, steps, periodic, bounce, **kw):
    phys = dict(tau_plus=0.9, magic=3 / 16, g=(1e-4, 3e-5, -2e-5))
    lat = L.Lattice(mask, bounce=bounce, periodic=periodic, **phys, **kw)
    lat.import_(f0)
    lat.step(steps)
    ref = O.run(mask, f0, steps, phys["tau_plus"], phys["magic"], phys["g"], BOUNCE[bounce],
                periodic=periodic)
    return lat, lat.export(), ref


@pytest.mark.parametrize("kw", FORMS)
@pytest.mark.parametrize("periodic", [0b000, 0b001, 0b110])
def test_halfway_wall_faces_random_state(L, kw, periodic):
    """Random solids, random populations and a 3-component force on a box
    whose rows span two workgroups with a ragged tail (70 nodes) and whose
    odd step count leaves the AA lattice in its reversed phase."""
    mask = I.random_solid_mask(70, 9, 11, seed=21, fraction=0.2)
    f0 = random_state(mask, seed=22, amplitude=0.02, bounce="halfway")
    lat, got, ref = _run(L, mask, f0, 11, periodic, "halfway", block=64, **kw)
    assert rel_maxabs(got, ref) <= TOL
    # the faces are walls: mass is conserved and the state differs from
    # the wrapped run
    assert abs(lat.macroscopic()["mass"] - f0.sum()) <= 1e-13 * f0.sum()
    wrapped = O.run(mask, f0, 11, 0.9, 3 / 16, (1e-4, 3e-5, -2e-5), 1)
    assert np.abs(wrapped - ref).max() > 1e-6


@pytest.mark.parametrize("kw", [{}, {"layout": "aos"}, {"propagation": "aa"},
                                {"propagation": "push"}, {"layout": "aos", "propagation": "push"}])
def test_fullway_solid_faces_equal_wrap(L, kw):
    """Full-way bounce-back with z not wrapping: the plates of the slab are
    the z boundary layers, and the run matches the oracle (which wraps the
    solid layers, as the library does)."""
    mask = I.slab_mask(40, 9, 12)
    f0 = random_state(mask, seed=23, amplitude=0.02, bounce="fullway")
    _, got, ref = _run(L, mask, f0, 10, 0b011, "fullway", **kw)
    assert rel_maxabs(got, ref) <= TOL


def test_fullway_open_face_refused(L):
    """A fluid node on a wall face cannot hold the populations full-way
    bounce-back stores: lbm_init_geometry refuses the box."""
    mask = I.slab_mask(8, 6, 7)
    with pytest.raises(L.LBMError):
        L.Lattice(mask, bounce="fullway", periodic="xz")


@pytest.mark.parametrize("storage,tol", [("f32s", 1e-6), ("f16sr", 2e-3)])
def test_wall_faces_shifted_storage(L, storage, tol):
    """The shifted storages on the same wall-face box: the flow part of the
    populations (f - w) against the FP64 oracle at their storage precision."""
    mask = I.random_solid_mask(70, 9, 11, seed=24, fraction=0.2)
    f0 = random_state(mask, seed=25, amplitude=0.02, bounce="halfway")
    lat, got, ref = _run(L, mask, f0, 11, 0b010, "halfway", storage=storage)
    _, w, _ = O.table()
    fl = mask.reshape(-1) == 0
    err = np.abs(got - ref)[fl].max() / np.abs(ref - w)[fl].max()
    assert err <= tol, err
