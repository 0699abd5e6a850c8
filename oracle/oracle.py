"""Python face of the reference oracle (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It loads ``lbm_oracle.c`` (plain C, double
precision, built with gcc and no floating-point contraction) through ctypes
and adds closed forms written from the mathematics:

* ``slab_profile``: steady force-driven flow between two plates normal to z
  (the verification set-up of the paper, Sect. 2.1), including the wall slip
  of TRT with mid-link bounce-back as a function of the magic parameter.
* ``duct_series``: steady flow through a rectangular duct, classical Fourier
  series of the Poisson problem.  It is not an exact solution of the
  discrete scheme; its use is convergence checks only.

Arrays cross the boundary in the canonical layout: populations
``f[N][19]`` float64 with node ``x + nx*(y + ny*z)``; masks ``uint8`` of
shape ``(nz, ny, nx)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liblbm_oracle.so")
_LIB_OMP = os.path.join(_BUILD, "liblbm_oracle_omp.so")

Q = 19
_libs = {}


def _build_one(out: str, extra, force: bool) -> str:
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", *extra, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return out


def build(force: bool = False, omp: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, no fast-math);
    ``omp``: the OpenMP build of the same source (used for timing on all
    cores; identical results).  ``force`` rebuilds both."""
    os.makedirs(_BUILD, exist_ok=True)
    serial = _build_one(_LIB, [], force)
    par = _build_one(_LIB_OMP, ["-fopenmp"], force) if (omp or force) else None
    return par if omp else serial


def _load(omp: bool = False):
    lib = _libs.get(omp)
    if lib is None:
        lib = ctypes.CDLL(build(omp=omp))
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        lib.ora_table.argtypes = [ip, dp, ip]
        lib.ora_equilibrium.argtypes = [ctypes.c_double, dp, dp]
        lib.ora_moments.argtypes = [dp, dp, dp, dp]
        lib.ora_collide_node.argtypes = [dp, dp, ctypes.c_double, ctypes.c_double, dp]
        lib.ora_tau_minus.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.ora_tau_minus.restype = ctypes.c_double
        lib.ora_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, u8p,
                                ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                dp, dp, ctypes.c_int]
        lib.ora_run.restype = ctypes.c_int
        lib.ora_run_box.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                    u8p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    dp, dp, ctypes.c_int]
        lib.ora_run_box.restype = ctypes.c_int
        lib.ora_macroscopic.argtypes = [ctypes.c_int64, u8p, dp, dp, dp, dp]
        lib.ora_rest_state.argtypes = [ctypes.c_int64, u8p, ctypes.c_int, dp]
        _libs[omp] = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def table():
    """(c[19][3] int, w[19] float64, opp[19] int) in the canonical order."""
    lib = _load()
    c = np.zeros(57, dtype=np.intc)
    w = np.zeros(19, dtype=np.float64)
    o = np.zeros(19, dtype=np.intc)
    lib.ora_table(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(w),
                  o.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return c.reshape(19, 3).astype(np.int64), w, o.astype(np.int64)


def equilibrium(rho: float, u) -> np.ndarray:
    e = np.zeros(19)
    uu = np.ascontiguousarray(u, dtype=np.float64)
    _load().ora_equilibrium(float(rho), _dp(uu), _dp(e))
    return e


def collide_node(f, g, tau_plus: float, magic: float) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.zeros(19)
    _load().ora_collide_node(_dp(f), _dp(g), tau_plus, magic, _dp(out))
    return out


def tau_minus(tau_plus: float, magic: float) -> float:
    return _load().ora_tau_minus(tau_plus, magic)


def rest_state(mask: np.ndarray, bounce: int) -> np.ndarray:
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    f = np.zeros((m.size, Q))
    _load().ora_rest_state(m.size, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                           bounce, _dp(f))
    return f


def run(mask: np.ndarray, f: np.ndarray, steps: int, tau_plus: float,
        magic: float, g, bounce: int, omp: bool = False, periodic: int = 7) -> np.ndarray:
    """Advance a copy of the canonical state ``f`` by ``steps`` updates.

    bounce: 0 = full-way, 1 = half-way.  ``omp``: run the OpenMP build
    (threads from OMP_NUM_THREADS; same results bit for bit).  ``periodic``:
    bit mask of the axes that wrap (bit 0 x, 1 y, 2 z); the faces of the
    others are walls (Sect. 3.2 periodicity, read per axis)."""
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = m.shape
    out = np.array(f, dtype=np.float64, order="C", copy=True).reshape(m.size, Q)
    gg = np.ascontiguousarray(g, dtype=np.float64)
    rc = _load(omp).ora_run_box(nx, ny, nz, periodic,
                                m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                bounce, tau_plus, magic, _dp(gg), _dp(out), steps)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def macroscopic(mask: np.ndarray, f: np.ndarray, g):
    """(rho[N], u[N][3]); solid nodes report zeros."""
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    f = np.ascontiguousarray(f, dtype=np.float64)
    rho = np.zeros(m.size)
    u = np.zeros((m.size, 3))
    gg = np.ascontiguousarray(g, dtype=np.float64)
    _load().ora_macroscopic(m.size, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            _dp(f), _dp(gg), _dp(rho), _dp(u))
    return rho, u


def residual(u_new: np.ndarray, u_old: np.ndarray, fluid: np.ndarray) -> float:
    """||u_new - u_old||_2 / ||u_new||_2 over fluid nodes, all components."""
    d = (u_new - u_old)[fluid]
    n = np.sqrt((u_new[fluid] ** 2).sum())
    return float(np.sqrt((d ** 2).sum()) / n) if n > 0 else float("inf")


def run_to_steady(mask, f, tau_plus, magic, g, bounce, tol, check_every=100,
                  max_steps=10_000_000, omp=False, periodic=7):
    """Iterate in chunks of ``check_every`` until the velocity residual
    between chunks falls below ``tol``.  Returns (f, steps, residual)."""
    fluid = np.asarray(mask).reshape(-1) == 0
    _, u_old = macroscopic(mask, f, g)
    steps = 0
    r = float("inf")
    while steps < max_steps:
        f = run(mask, f, check_every, tau_plus, magic, g, bounce, omp=omp, periodic=periodic)
        steps += check_every
        _, u = macroscopic(mask, f, g)
        r = residual(u, u_old, fluid)
        u_old = u
        if r < tol:
            break
    return f, steps, r


def slab_profile(nz: int, tau_plus: float, magic: float, gx: float) -> np.ndarray:
    """Steady u_x(z) between plates at z = 0 and z = nz-1 (solid layers).

    Fluid layers z = 1..N with N = nz-2; mid-link walls at z = 1/2 and
    N + 1/2, centred coordinate zeta = z - (nz-1)/2.  The continuum parabola
    is (g/2nu)[(N/2)^2 - zeta^2]; TRT with mid-link bounce-back adds the
    uniform slip g(16 Lambda - 3)/(24 nu), which vanishes at Lambda = 3/16.
    Solid layers report 0."""
    nu = (tau_plus - 0.5) / 3.0
    n_fl = nz - 2
    zeta = np.arange(nz) - (nz - 1) / 2.0
    u = gx / (2.0 * nu) * ((n_fl / 2.0) ** 2 - zeta ** 2) + gx * (16.0 * magic - 3.0) / (24.0 * nu)
    u[0] = 0.0
    u[-1] = 0.0
    return u


def slab_parabola(nz: int, nu: float, gx: float) -> np.ndarray:
    """Continuum Poiseuille parabola with walls half a node outside the
    outermost fluid layers (no slip term); zero on the solid layers."""
    n_fl = nz - 2
    zeta = np.arange(nz) - (nz - 1) / 2.0
    u = gx / (2.0 * nu) * ((n_fl / 2.0) ** 2 - zeta ** 2)
    u[0] = 0.0
    u[-1] = 0.0
    return u


def duct_series(ny: int, nz: int, nu: float, gx: float, terms: int = 201) -> np.ndarray:
    """Steady u_x(y, z) in a duct with solid layers y in {0, ny-1},
    z in {0, nz-1} and mid-link walls: half-widths a = (ny-2)/2 (y) and
    b = (nz-2)/2 (z).  Solves nu (u_yy + u_zz) = -g with u = 0 on the walls
    by the series over odd n of cos(n pi y / 2a) modes.  Returns [nz][ny]."""
    a = (ny - 2) / 2.0
    b = (nz - 2) / 2.0
    y = np.arange(ny) - (ny - 1) / 2.0
    z = np.arange(nz) - (nz - 1) / 2.0
    Y, Z = np.meshgrid(y, z)  # shape (nz, ny)
    u = np.zeros_like(Y)
    for n in range(1, terms + 1, 2):
        k = n * np.pi / (2.0 * a)
        sign = 1.0 if ((n - 1) // 2) % 2 == 0 else -1.0
        # cosh ratio written with exponentials of non-positive arguments
        ratio = (np.exp(k * (np.abs(Z) - b)) + np.exp(-k * (np.abs(Z) + b))) / (1.0 + np.exp(-2.0 * k * b))
        u += sign / n ** 3 * (1.0 - ratio) * np.cos(k * Y)
    u *= 16.0 * a * a * gx / (nu * np.pi ** 3)
    u[:, 0] = u[:, -1] = 0.0
    u[0, :] = u[-1, :] = 0.0
    return u


def time_run(mask, steps, tau_plus, magic, g, bounce, omp=False):
    """Wall-clock seconds of ``steps`` oracle updates from the rest state
    (single thread, or the OpenMP build with OMP_NUM_THREADS threads).
    Used for the CPU baseline figure."""
    f = rest_state(mask, bounce)
    t0 = time.perf_counter()
    run(mask, f, steps, tau_plus, magic, g, bounce, omp=omp)
    return time.perf_counter() - t0
