"""The n-asset generalisation, Eq. (bse_general) (Sec. 3.2), for three assets,
in FP64 (TEST INFRASTRUCTURE ONLY).

Only tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py may
import this module; it shares no code with the HIP library.

In time to maturity tau = T - t, Eq. (bse_general) reads

    u_tau = 1/2 sum_{d,e} rho_de s_d s_e x_d x_e u_{x_d x_e} + r sum_d x_d u_{x_d} - r u,

with rho_dd = 1.  On the uniform grid x_d = k_d h of M nodes per axis on
[0, s_max]^3 the centred differences of Eq. (fd) give, in index form (h
cancels),

    L_h u = sum_d a_d (u[+d] - 2u + u[-d])
          + sum_{d<e} g_de (u[+d+e] + u[-d-e] - u[+d-e] - u[-d+e])
          + sum_d m_d (u[+d] - u[-d]) - r u,

    a_d = s_d^2 k_d^2 / 2,  g_de = rho_de s_d s_e k_d k_e / 4,  m_d = r k_d / 2,

where u[+d] is the neighbour one node up along axis d.  The symmetric sum over
d != e counts each pair twice, which turns the 1/2 into the full rho_de s_d s_e
x_d x_e, and the four-corner difference divided by 4 h^2 is the mixed
derivative: hence g_de.  The stencil has 1 + 6 + 12 = 19 points.

Time stepping is explicit Euler (the explicit reading of the fine propagator
used throughout the two-asset path), the Dirichlet faces hold the forward
intrinsic value max(w . S - K e^{-r tau}, 0) of the basket call
max(w . S - K, 0) at every step; where the max is active this is an exact
solution of the PDE (second derivatives vanish, the drift and the discount
cancel).  The numerical coarse propagator is the same scheme on a coarser grid
with injection and trilinear prolongation, its output faces overwritten with
the fine boundary data, as in the two-asset path.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

PAIRS = ((0, 1), (0, 2), (1, 2))


@dataclass(frozen=True)
class Problem3:
    """M^3 nodes on [0, s_max]^3; sigma = (s1, s2, s3); rho = (rho12, rho13, rho23)."""
    M: int
    sigma: tuple
    rho: tuple
    r: float
    w: tuple = (1 / 3, 1 / 3, 1 / 3)
    strike: float = 1.0
    s_max: float = 4.0

    def with_M(self, M: int) -> "Problem3":
        return Problem3(M, self.sigma, self.rho, self.r, self.w, self.strike, self.s_max)


def coords(p: Problem3) -> np.ndarray:
    return np.arange(p.M) * (p.s_max / (p.M - 1))


def _mesh(p: Problem3):
    x = coords(p)
    return np.meshgrid(x, x, x, indexing="ij")


def payoff_grid(p: Problem3) -> np.ndarray:
    """max(w . S - K, 0) on every node (Sec. 3.2's terminal condition, basket form)."""
    X = _mesh(p)
    return np.maximum(sum(p.w[d] * X[d] for d in range(3)) - p.strike, 0.0)


def boundary_grid(p: Problem3, tau: float) -> np.ndarray:
    """max(w . S - K e^{-r tau}, 0) on every node (only the faces are used)."""
    X = _mesh(p)
    return np.maximum(sum(p.w[d] * X[d] for d in range(3)) - p.strike * math.exp(-p.r * tau), 0.0)


def _shift(u: np.ndarray, off) -> np.ndarray:
    """u at interior node + off (off a 3-tuple of -1/0/1): an (M-2)^3 view."""
    M = u.shape[0]
    return u[1 + off[0]:M - 1 + off[0], 1 + off[1]:M - 1 + off[1], 1 + off[2]:M - 1 + off[2]]


def _unit(d: int, s: int):
    o = [0, 0, 0]
    o[d] = s
    return tuple(o)


def _two(d: int, sd: int, e: int, se: int):
    o = [0, 0, 0]
    o[d] = sd
    o[e] = se
    return tuple(o)


def apply_operator(p: Problem3, u: np.ndarray) -> np.ndarray:
    """L_h u at the interior nodes, shape (M-2)^3, term by term as written above."""
    k = np.arange(1, p.M - 1, dtype=np.float64)
    K = np.meshgrid(k, k, k, indexing="ij")
    c = _shift(u, (0, 0, 0))
    out = -p.r * c
    for d in range(3):
        a = 0.5 * p.sigma[d] ** 2 * K[d] ** 2
        m = 0.5 * p.r * K[d]
        up, dn = _shift(u, _unit(d, 1)), _shift(u, _unit(d, -1))
        out = out + a * (up - 2.0 * c + dn) + m * (up - dn)
    for (d, e), rho in zip(PAIRS, p.rho):
        g = 0.25 * rho * p.sigma[d] * p.sigma[e] * K[d] * K[e]
        out = out + g * (_shift(u, _two(d, 1, e, 1)) + _shift(u, _two(d, -1, e, -1))
                         - _shift(u, _two(d, 1, e, -1)) - _shift(u, _two(d, -1, e, 1)))
    return out


def euler_step(p: Problem3, dt: float, u: np.ndarray, faces: np.ndarray) -> np.ndarray:
    """u + dt L_h u inside; the faces (boundary nodes) taken from `faces`."""
    out = np.array(faces, dtype=np.float64, copy=True)
    out[1:-1, 1:-1, 1:-1] = u[1:-1, 1:-1, 1:-1] + dt * apply_operator(p, u)
    return out


def fine(p: Problem3, m: int, dt: float, tau0: float, u: np.ndarray, faces=None) -> np.ndarray:
    """m explicit steps of dt from tau0; faces(p, tau) gives the boundary data
    (default: the forward intrinsic value)."""
    faces = faces or boundary_grid
    for q in range(m):
        u = euler_step(p, dt, u, faces(p, tau0 + (q + 1) * dt))
    return u


def stable_dt(p: Problem3) -> float:
    """Gershgorin bound of explicit Euler, 2 / max_row (|diag| + sum |off|),
    with the diagonal -(2 sum a_d + r) and the off-diagonals a_d +- m_d and
    the four +-g_de of every pair, maximised over the interior rows."""
    k = np.arange(1, p.M - 1, dtype=np.float64)
    K = np.meshgrid(k, k, k, indexing="ij")
    diag = np.full(K[0].shape, p.r)
    off = np.zeros(K[0].shape)
    for d in range(3):
        a = 0.5 * p.sigma[d] ** 2 * K[d] ** 2
        m = 0.5 * p.r * K[d]
        diag = diag + 2.0 * a
        off = off + np.abs(a + m) + np.abs(a - m)
    for (d, e), rho in zip(PAIRS, p.rho):
        off = off + 4.0 * np.abs(0.25 * rho * p.sigma[d] * p.sigma[e] * K[d] * K[e])
    return 2.0 / float(np.max(np.abs(diag) + off))


def steps_for(p: Problem3, dT: float, cfl: float = 0.9) -> int:
    return int(math.ceil(dT / (cfl * stable_dt(p)) - 1e-12))


def restrict(u: np.ndarray, q: int) -> np.ndarray:
    """Injection at the coincident nodes (every q-th node on each axis)."""
    return np.ascontiguousarray(u[::q, ::q, ::q])


def prolong(c: np.ndarray, q: int) -> np.ndarray:
    """Trilinear interpolation from the coarse nodes to the fine grid."""
    Mc = c.shape[0]
    Mf = (Mc - 1) * q + 1
    t = np.arange(Mf) / q
    i0 = np.minimum(np.floor(t).astype(int), Mc - 2)
    f = t - i0
    out = np.zeros((Mf, Mf, Mf))
    for a in (0, 1):
        wa = f if a else 1.0 - f
        for b in (0, 1):
            wb = f if b else 1.0 - f
            for cc in (0, 1):
                wc = f if cc else 1.0 - f
                out += (wa[:, None, None] * wb[None, :, None] * wc[None, None, :]
                        * c[np.ix_(i0 + a, i0 + b, i0 + cc)])
    return out


def coarse(pf: Problem3, Mc: int, m: int, dt: float, tau0: float, u: np.ndarray) -> np.ndarray:
    """Numerical G over one slice: restrict, m explicit steps on the Mc^3 grid,
    prolong, faces set to the fine boundary data at the slice end."""
    q = (pf.M - 1) // (Mc - 1)
    pc = pf.with_M(Mc)
    c = fine(pc, m, dt, tau0, restrict(u, q))
    out = prolong(c, q)
    faces = boundary_grid(pf, tau0 + m * dt)
    out[0, :, :], out[-1, :, :] = faces[0, :, :], faces[-1, :, :]
    out[:, 0, :], out[:, -1, :] = faces[:, 0, :], faces[:, -1, :]
    out[:, :, 0], out[:, :, -1] = faces[:, :, 0], faces[:, :, -1]
    return out


def serial_fine(p: Problem3, N: int, T: float, m: int) -> np.ndarray:
    dT = T / N
    u = payoff_grid(p)
    for n in range(N):
        u = fine(p, m, dT / m, n * dT, u)
    return u
