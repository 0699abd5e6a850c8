"""The pins are sharp: each planted mistake in the oracle fails at least one.

Every case below copies ``oracle/lbm_oracle.c`` to a temporary directory,
plants one plausible mistake (a dropped or wrong term, a wrong sign, index
or rate), builds it with gcc and runs the fast pins of
``test_oracle_pins.py`` against the mutant.  The committed oracle is never
modified; everything runs on the CPU.
"""
import ctypes
import os
import subprocess

import pytest

from oracle import oracle as O
import tests.test_oracle_pins as P

SRC = os.path.join(os.path.dirname(O.__file__), "lbm_oracle.c")

MUTATIONS = {
    "eq_quadratic_coeff": ("4.5 * cu * cu", "4.0 * cu * cu"),
    "eq_uu_coeff": ("- 1.5 * uu", "- 1.0 * uu"),
    "velocity_half_force_shift": ("(j[a] + 0.5 * g[a])", "(j[a] + g[a])"),
    "force_sign": ("3.0 * (ORA_C[i][a] - u[a])", "3.0 * (ORA_C[i][a] + u[a])"),
    "force_symmetric_prefactor": ("(1.0 - 0.5 * lp) * Fp", "(1.0 - lp) * Fp"),
    "antisymmetric_rate": ("double lm = 1.0 / ora_tau_minus(tau_plus, magic);",
                           "double lm = lp;"),
    "tau_minus_formula": ("return 0.5 + magic / (tau_plus - 0.5);",
                          "return 0.5 + magic * (tau_plus - 0.5);"),
    "stream_direction": ("int64_t tx = x + ORA_C[i][0],", "int64_t tx = x - ORA_C[i][0],"),
    "wall_face_ignored_on_x": ("int beyond = ora_outside(tx, nx, periodic, 0) ||",
                               "int beyond = 0 * ora_outside(tx, nx, periodic, 0) ||"),
    "wall_face_wrong_axis_bit": ("return !((periodic >> axis) & 1u)", "return !((periodic >> 0) & 1u)"),
    "wall_face_off_by_one": ("(v < 0 || v >= n)", "(v < 0 || v > n)"),
    "halfway_reflect_index": ("f[ORA_Q * n + ora_opposite(i)] = post[ORA_Q * n + i];",
                              "f[ORA_Q * n + i] = post[ORA_Q * n + i];"),
    "fullway_no_reversal": ("pn[i] = fn[ora_opposite(i)];", "pn[i] = fn[i];"),
    "table_diagonal_sign": ("{1, -1, 0},  {-1, 1, 0},", "{1, 1, 0},  {-1, 1, 0},"),
    "diagonal_weight": ("return 1.0 / 36.0;", "return 1.0 / 37.0;"),
}

FAST_PINS = [
    (P.test_table_isotropy_exact, {}),
    (P.test_equilibrium_moments, {}),
    (P.test_collision_moments, {"tau_plus": 0.8, "magic": 3 / 16}),
    (P.test_uniform_equilibrium_invariant, {"bounce": 0}),
    (P.test_mass_conserved, {"bounce": 0}),
    (P.test_mass_conserved, {"bounce": 1}),
    (P.test_momentum_grows_by_force, {}),
    (P.test_slab_closed_form, {"magic": 1 / 4, "bounce": 0}),
    (P.test_slab_closed_form, {"magic": 1 / 4, "bounce": 1}),
    (P.test_brute_force_4cubed, {"bounce": 0}),
    (P.test_brute_force_4cubed, {"bounce": 1}),
    (P.test_brute_force_wall_faces, {"periodic": 0b001}),
    (P.test_brute_force_wall_faces, {"periodic": 0b110}),
    (P.test_wall_faces_equal_solid_layers, {"periodic": 0b101}),
]


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, "mutation anchor missing: %s" % name
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new, 1))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                           "-ffp-contract=off", "-o", str(so), str(mutant), "-lm"])
    real = O._load()  # the real library, whose argtypes are set
    lib = ctypes.CDLL(str(so))
    for fn in ("ora_table", "ora_equilibrium", "ora_moments", "ora_collide_node",
               "ora_tau_minus", "ora_run", "ora_run_box", "ora_macroscopic", "ora_rest_state"):
        getattr(lib, fn).argtypes = getattr(real, fn).argtypes
        getattr(lib, fn).restype = getattr(real, fn).restype
    monkeypatch.setitem(O._libs, False, lib)
    failed = []
    for fn, kw in FAST_PINS:
        try:
            fn(**kw)
        except (AssertionError, ValueError, FloatingPointError, KeyError, IndexError):
            failed.append(fn.__name__)
            # one catch suffices; a mutant with a broken table can also
            # index out of bounds, so it is run no further than needed
            break
    assert failed, "no pin caught the planted mistake %s" % name
