"""FP64 CPU oracle for Parareal on the two-asset Black-Scholes equation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library under ``paper_2404_02521_amd/`` and never imports
it.

* ``bs2d.c`` (built into ``liboracle.so`` by :func:`build`) holds the grid,
  the Dirichlet data, the explicit finite-difference propagator of Eq. (fd)
  (Sec. 3.2, explicit instead of implicit Euler), the numerical coarse
  propagator and Eq. (parareal) (Sec. 3.1).
* :mod:`oracle.closed_forms` holds Margrabe's formula and the one-asset
  Black-Scholes call, written independently of ``bs2d.c``.
* :mod:`oracle.fno` holds the Fourier neural operator of Sec. 3.4 in NumPy
  FP64 with hand-derived gradients.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bs2d.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

PAYOFF_BASKET = 0
PAYOFF_EXCHANGE = 1
BC_FORWARD_INTRINSIC = 0
BC_DISCOUNTED_PAYOFF = 1
BC_EXACT = 2
G_NUMERICAL = 0
G_FINE = 1
G_LOD = 2


def build(force: bool = True) -> str:
    """Compile ``bs2d.c`` with gcc into ``liboracle.so`` (plain IEEE FP64)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(C.Structure):
    _fields_ = [("M", C.c_int32), ("payoff_kind", C.c_int32), ("bc_kind", C.c_int32),
                ("pad_", C.c_int32), ("s_max", C.c_double), ("sigma1", C.c_double),
                ("sigma2", C.c_double), ("rho", C.c_double), ("r", C.c_double),
                ("w1", C.c_double), ("w2", C.c_double), ("strike", C.c_double)]


@dataclass(frozen=True)
class Problem:
    """Grid + model + payoff: M x M nodes on [0, s_max]^2 (both boundaries)."""
    M: int
    sigma1: float
    sigma2: float
    rho: float
    r: float
    payoff_kind: int = PAYOFF_BASKET
    w1: float = 0.5
    w2: float = 0.5
    strike: float = 1.0
    bc_kind: int = BC_FORWARD_INTRINSIC
    s_max: float = 4.0

    def with_M(self, M: int) -> "Problem":
        d = dict(self.__dict__)
        d["M"] = M
        return Problem(**d)

    def c(self) -> _Problem:
        return _Problem(self.M, self.payoff_kind, self.bc_kind, 0, self.s_max, self.sigma1,
                        self.sigma2, self.rho, self.r, self.w1, self.w2, self.strike)

    @property
    def h(self) -> float:
        return self.s_max / (self.M - 1)


_PROP = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double))
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER(_Problem)
        D = C.POINTER(C.c_double)
        sig = {
            "orc_payoff": (C.c_double, [P, C.c_double, C.c_double]),
            "orc_bc": (C.c_double, [P, C.c_double, C.c_double, C.c_double]),
            "orc_margrabe": (C.c_double, [C.c_double] * 6),
            "orc_bs_call": (C.c_double, [C.c_double] * 5),
            "orc_init": (None, [P, D]),
            "orc_set_boundary": (None, [P, C.c_double, D]),
            "orc_apply_operator": (None, [P, D, D]),
            "orc_euler_step": (None, [P, C.c_double, D, D]),
            "orc_fine": (None, [P, C.c_int, C.c_double, C.c_double, D, D]),
            "orc_stable_dt": (C.c_double, [P]),
            "orc_steps_for": (C.c_int32, [P, C.c_double, C.c_double]),
            "orc_restrict": (None, [C.c_int, C.c_int, D, D]),
            "orc_prolong": (None, [C.c_int, C.c_int, D, D]),
            "orc_coarse": (None, [P, P, C.c_int, C.c_double, C.c_double, D, D]),
            "orc_parareal": (C.c_int32, [C.c_int64, C.c_int32, D, _PROP, C.c_void_p, _PROP,
                                         C.c_void_p, C.c_int32, C.c_double, C.c_int32, D, D]),
            "orc_serial_fine": (None, [P, C.c_int32, C.c_double, C.c_int32, D]),
            "orc_parareal_bs": (C.c_int32, [P, P, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                            C.c_int32, C.c_int32, C.c_double, C.c_int32, D, D]),
            "orc_num_threads": (C.c_int32, []),
            "orc_lod_step_ring": (None, [P, C.c_double, D, D, D]),
            "orc_lod": (None, [P, C.c_int, C.c_double, C.c_double, D, D]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _grid(p: Problem, u=None) -> np.ndarray:
    if u is None:
        return np.zeros((p.M, p.M), dtype=np.float64)
    return np.ascontiguousarray(u, dtype=np.float64).reshape(p.M, p.M).copy()


def coords(p: Problem) -> np.ndarray:
    """Node coordinates x_i = i * h (the same for both axes)."""
    return np.arange(p.M, dtype=np.float64) * p.h


def payoff_grid(p: Problem) -> np.ndarray:
    u = _grid(p)
    pc = p.c()
    lib().orc_init(C.byref(pc), _dp(u))
    return u


def bc(p: Problem, x: float, y: float, tau: float) -> float:
    pc = p.c()
    return lib().orc_bc(C.byref(pc), x, y, tau)


def set_boundary(p: Problem, tau: float, u: np.ndarray) -> np.ndarray:
    u = _grid(p, u)
    pc = p.c()
    lib().orc_set_boundary(C.byref(pc), tau, _dp(u))
    return u


def apply_operator(p: Problem, u: np.ndarray) -> np.ndarray:
    """L_h u at interior nodes (boundary entries zero)."""
    u = _grid(p, u)
    out = _grid(p)
    pc = p.c()
    lib().orc_apply_operator(C.byref(pc), _dp(u), _dp(out))
    return out


def euler_step(p: Problem, dt: float, u: np.ndarray) -> np.ndarray:
    """u + dt L_h u at interior nodes; the ring is copied from u unchanged."""
    u = _grid(p, u)
    out = u.copy()
    pc = p.c()
    lib().orc_euler_step(C.byref(pc), dt, _dp(u), _dp(out))
    return out


def fine(p: Problem, m: int, dt: float, tau0: float, u: np.ndarray) -> np.ndarray:
    u = _grid(p, u)
    pc = p.c()
    lib().orc_fine(C.byref(pc), m, dt, tau0, _dp(u), _dp(u))
    return u


def stable_dt(p: Problem) -> float:
    pc = p.c()
    return lib().orc_stable_dt(C.byref(pc))


def steps_for(p: Problem, dT: float, cfl: float) -> int:
    pc = p.c()
    return int(lib().orc_steps_for(C.byref(pc), dT, cfl))


def restrict(Mf: int, Mc: int, u: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros((Mc, Mc))
    lib().orc_restrict(Mf, Mc, _dp(u), _dp(out))
    return out


def prolong(Mc: int, Mf: int, c: np.ndarray) -> np.ndarray:
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros((Mf, Mf))
    lib().orc_prolong(Mc, Mf, _dp(c), _dp(out))
    return out


def coarse(pf: Problem, pc_: Problem, m: int, dt: float, tau0: float, u: np.ndarray) -> np.ndarray:
    u = _grid(pf, u)
    out = _grid(pf)
    a, b = pf.c(), pc_.c()
    lib().orc_coarse(C.byref(a), C.byref(b), m, dt, tau0, _dp(u), _dp(out))
    return out


def lod_step_ring(p: Problem, dt: float, u: np.ndarray, ring1: np.ndarray) -> np.ndarray:
    """One locally one-dimensional implicit step; ring1's ring = values at the new time."""
    u = _grid(p, u)
    ring1 = _grid(p, ring1)
    out = _grid(p)
    pc = p.c()
    lib().orc_lod_step_ring(C.byref(pc), dt, _dp(u), _dp(ring1), _dp(out))
    return out


def lod(p: Problem, m: int, dt: float, tau0: float, u: np.ndarray) -> np.ndarray:
    """Same-grid coarse propagator: m LOD implicit steps from tau0."""
    u = _grid(p, u)
    out = _grid(p)
    pc = p.c()
    lib().orc_lod(C.byref(pc), m, dt, tau0, _dp(u), _dp(out))
    return out


def serial_fine(p: Problem, N: int, T: float, mF: int) -> np.ndarray:
    out = _grid(p)
    pc = p.c()
    lib().orc_serial_fine(C.byref(pc), N, T, mF, _dp(out))
    return out


def parareal_bs(pf: Problem, pc_: Problem, N: int, T: float, mF: int, mG: int,
                coarse_kind: int = G_NUMERICAL, max_iters: int | None = None, tol: float = 1e-8,
                tol_relative: bool = False):
    """Eq. (parareal) on the Black-Scholes problem.  Returns (U^K_N, K, increments)."""
    out = _grid(pf)
    inc = np.zeros(N + 1)
    a, b = pf.c(), pc_.c()
    K = lib().orc_parareal_bs(C.byref(a), C.byref(b), N, T, mF, mG, coarse_kind,
                              N if max_iters is None else max_iters, tol, int(tol_relative),
                              _dp(out), _dp(inc))
    if K < 0:
        raise FloatingPointError("oracle Parareal: non-finite increment")
    return out, int(K), inc[:K].copy()


def parareal_generic(u0: np.ndarray, N: int, F, G, max_iters: int, tol: float = 0.0,
                     tol_relative: bool = False):
    """The C Parareal driver with Python propagators F(n, x) -> y, G(n, x) -> y.

    Returns (U, K, increments) with U of shape (N+1, len)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64).ravel()
    L = u0.size

    def wrap(fn):
        def cb(_ctx, n, pin, pout):
            x = np.ctypeslib.as_array(pin, shape=(L,)).copy()
            y = np.asarray(fn(int(n), x), dtype=np.float64).ravel()
            np.ctypeslib.as_array(pout, shape=(L,))[:] = y
        return _PROP(cb)

    cf, cg = wrap(F), wrap(G)
    U = np.zeros((N + 1, L))
    inc = np.zeros(N + 1)
    K = lib().orc_parareal(L, N, _dp(u0), cf, None, cg, None, max_iters, tol, int(tol_relative),
                           _dp(U), _dp(inc))
    if K < 0:
        raise FloatingPointError("oracle Parareal: non-finite increment")
    return U, int(K), inc[:K].copy()


def num_threads() -> int:
    return int(lib().orc_num_threads())
