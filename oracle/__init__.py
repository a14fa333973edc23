"""FP64 CPU oracle of the exponential-integrator PIC step.

TEST INFRASTRUCTURE ONLY: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library and never imports it.

Layout:
  ``pic_oracle.c``  plain C, FP64: CIC deposit, trapezoid Poisson solve, CIC
                    gather, potential, Strang / ETD1 / ETD2RK pushes, moments,
                    whole runs (ctypes bindings below)
  ``fine_oracle.c`` plain C, FP64: the paper's reference RK4 solver (field
                    re-solved at every stage), its improved ETD scheme
                    (Algorithm 3.4: periods, N_i, o_i, interpolation,
                    extrapolation) and the classic / modified ETD scheme
                    (Algorithm 2.1 with 2 pi eps or the mean period)
  ``duffing.py``    exact Duffing solution by Jacobi elliptic functions and the
                    paper's period formulas (appendix A)
  ``mlp.py``        FP64 forward/backward of the learned corrector network

Parity unpinned: nothing here (every function has a pin in tests/test_oracle_*.py).
"""
import ctypes
import os

import numpy as np

from . import build as _build

FIELD_ZERO, FIELD_DUFFING, FIELD_POISSON, FIELD_CONST = 0, 1, 2, 3
SCHEME_STRANG, SCHEME_ETD1, SCHEME_ETD2RK = 0, 1, 2
MOMENT_NAMES = ("charge", "rms_radius", "energy", "kinetic", "potential", "n_offmesh", "n_nan")

_lib = None


def lib():
    """Load (building first if absent or stale) the C oracle."""
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        p = ctypes.POINTER(ctypes.c_double)
        L.orc_deposit.argtypes = [p, i64, d, i32, d, d, p]
        L.orc_deposit.restype = i64
        L.orc_set_threads.argtypes = [i32]
        L.orc_set_threads.restype = None
        L.orc_poisson.argtypes = [p, i32, d, d, p, p, p]
        L.orc_poisson.restype = None
        L.orc_gather.argtypes = [d, p, d, i32, d, d]
        L.orc_gather.restype = d
        L.orc_potential.argtypes = [d, p, p, d, i32, d, d]
        L.orc_potential.restype = d
        L.orc_push.argtypes = [p, p, i64, d, d, i32, i32, i32, p, d, i32, d, d, d]
        L.orc_push.restype = None
        L.orc_moments.argtypes = [p, p, i64, d, d, i32, p, i32, d, d, p]
        L.orc_moments.restype = None
        L.orc_run.argtypes = [p, p, i64, d, d, d, i32, i32, i32, i64, i32, d, d, d, p]
        L.orc_run.restype = None
        L.orc_rk4_run.argtypes = [p, p, i64, d, d, d, i64, i32, d, i32, d, d]
        L.orc_rk4_run.restype = i32
        L.orc_improved_etd_step.argtypes = [p, p, i64, d, d, d, d, i32, d, i32, d, d, i64, i32,
                                            p, ctypes.POINTER(ctypes.c_int64), d]
        L.orc_improved_etd_step.restype = i64
        L.orc_classic_etd_step.argtypes = [p, p, i64, d, d, d, d, i32, d, i32, d, d, i32, i64,
                                           p, p]
        L.orc_classic_etd_step.restype = i64
        L.orc_threads.argtypes = []
        L.orc_threads.restype = i32
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def deposit(R, w, nr, rmin, rmax):
    """CIC charge density on the nr+1 nodes; returns (rho, n_offmesh)."""
    R = _f64(R)
    rho = np.zeros(nr + 1)
    off = lib().orc_deposit(_ptr(R), R.size, w, nr, rmin, rmax, _ptr(rho))
    return rho, int(off)


def poisson(rho, nr, rmin, rmax):
    """Trapezoid Poisson solve; returns (E, Psi, Qb)."""
    rho = _f64(rho)
    E = np.zeros(nr + 1)
    Psi = np.zeros(nr + 1)
    Qb = ctypes.c_double(0.0)
    lib().orc_poisson(_ptr(rho), nr, rmin, rmax, _ptr(E), _ptr(Psi), ctypes.byref(Qb))
    return E, Psi, Qb.value


def gather(R, E, Qb, nr, rmin, rmax):
    E = _f64(E)
    L = lib()
    return np.array([L.orc_gather(float(r), _ptr(E), Qb, nr, rmin, rmax) for r in np.ravel(R)])


def potential(R, E, Psi, Qb, nr, rmin, rmax):
    E = _f64(E)
    Psi = _f64(Psi)
    L = lib()
    return np.array([L.orc_potential(float(r), _ptr(E), _ptr(Psi), Qb, nr, rmin, rmax)
                     for r in np.ravel(R)])


def push(R, V, dt, eps, K, scheme=SCHEME_STRANG, field=FIELD_DUFFING, E=None, Qb=0.0,
         nr=0, rmin=0.0, rmax=0.0, E0=0.0):
    """One macro step in a frozen field; returns new (R, V) copies."""
    R = _f64(R).copy()
    V = _f64(V).copy()
    E = None if E is None else _f64(E)
    lib().orc_push(_ptr(R), _ptr(V), R.size, dt, eps, K, scheme, field, _ptr(E), Qb, nr,
                   rmin, rmax, E0)
    return R, V


def moments(R, V, w, eps, field, E=None, nr=0, rmin=0.0, rmax=0.0):
    R = _f64(R)
    V = _f64(V)
    E = None if E is None else _f64(E)
    out = np.zeros(7)
    lib().orc_moments(_ptr(R), _ptr(V), R.size, w, eps, field, _ptr(E), nr, rmin, rmax,
                      _ptr(out))
    return dict(zip(MOMENT_NAMES, out))


def run(R, V, w, dt, eps, K, n_steps, field, scheme=SCHEME_STRANG, nr=0, rmin=0.0,
        rmax=0.0, E0=0.0, with_moments=False):
    """n_steps PIC steps.  Returns (R, V) or (R, V, moments[n_steps+1, 7])."""
    R = _f64(R).copy()
    V = _f64(V).copy()
    mom = np.zeros((n_steps + 1, 7)) if with_moments else None
    lib().orc_run(_ptr(R), _ptr(V), R.size, w, dt, eps, K, scheme, field, n_steps, nr, rmin,
                  rmax, E0, _ptr(mom))
    if with_moments:
        return R, V, mom
    return R, V


def rk4_run(R, V, w, eps, h, n_steps, field, nr=0, rmin=0.0, rmax=0.0, E0=0.0):
    """n_steps of the reference RK4 solver (step h); returns new (R, V)."""
    R = _f64(R).copy()
    V = _f64(V).copy()
    if lib().orc_rk4_run(_ptr(R), _ptr(V), R.size, w, eps, h, n_steps, field, E0, nr, rmin,
                         rmax) != 0:
        raise MemoryError("orc_rk4_run")
    return R, V


def fine_step(eps):
    """The paper's reference step 2 pi eps / 100."""
    return 2.0 * np.pi * eps / 100.0


def improved_etd_step(R, V, w, dt, eps, field, nr=0, rmin=0.0, rmax=0.0, E0=0.0, h=None,
                      max_fine=100000, T=None, alt_window=0.0):
    """One macro step of Algorithm 3.4.  Returns (R, V, T, N, n_unresolved).
    With T given (the periods of a previous step, in the given field where
    they are constant) the period search is skipped.  With alt_window > 0,
    particles whose dt / T_i is within alt_window of a whole number take the
    other valid split of dt into whole periods and a remainder (N_i one
    smaller or larger), the outcome a computation whose T_i differs by a
    rounding may choose there."""
    R = _f64(R).copy()
    V = _f64(V).copy()
    h = fine_step(eps) if h is None else h
    given = T is not None
    T = _f64(T).copy() if given else np.empty(R.size)
    N = np.empty(R.size, dtype=np.int64)
    un = lib().orc_improved_etd_step(_ptr(R), _ptr(V), R.size, w, dt, eps, h, field, E0, nr,
                                     rmin, rmax, max_fine, 1 if given else 0, _ptr(T),
                                     N.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     float(alt_window))
    if un < 0:
        raise MemoryError("orc_improved_etd_step")
    return R, V, T, N, int(un)


def classic_etd_step(R, V, w, dt, eps, field, modified, nr=0, rmin=0.0, rmax=0.0, E0=0.0,
                     h=None, max_fine=100000):
    """One macro step of Algorithm 2.1 with the period 2 pi eps (modified =
    False) or the particles' mean period (modified = True).
    Returns (R, V, P, T, n_unresolved); T is the periods (modified) or None."""
    R = _f64(R).copy()
    V = _f64(V).copy()
    h = fine_step(eps) if h is None else h
    T = np.empty(R.size)
    P = ctypes.c_double(0.0)
    un = lib().orc_classic_etd_step(_ptr(R), _ptr(V), R.size, w, dt, eps, h, field, E0, nr, rmin,
                                    rmax, 1 if modified else 0, max_fine, _ptr(T),
                                    ctypes.byref(P))
    if un < 0:
        raise MemoryError("orc_classic_etd_step")
    return R, V, P.value, (T if modified else None), int(un)


def threads():
    return int(lib().orc_threads())


def set_threads(n):
    """OpenMP threads of later pushes (timing only; results do not depend on it)."""
    lib().orc_set_threads(int(n))
