"""Implicit-Euler fine propagator of Eq. (fd) in FP64 (TEST INFRASTRUCTURE ONLY).

Only tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py may
import this module; it shares no code with the HIP library.

Eq. (fd) (Sec. 3.2) is implicit Euler in time with the centred nine-point
operator in space: every step solves

    u^{m+1}_{ij} - dt L_h u^{m+1}_{ij} = u^m_{ij}      at every interior node,

with the Dirichlet ring of u^{m+1} set to the boundary data at tau^{m+1}.  In
index form (x_i = i h, h cancels) the row of node (i, j) is

    (1 + dt (2 alpha + 2 beta + r)) u_ij
      - dt (alpha + mu) u_{i+1,j} - dt (alpha - mu) u_{i-1,j}
      - dt (beta + nu) u_{i,j+1}  - dt (beta - nu) u_{i,j-1}
      - dt gamma (u_{i+1,j+1} + u_{i-1,j-1} - u_{i+1,j-1} - u_{i-1,j+1})

with alpha = s1^2 i^2 / 2, beta = s2^2 j^2 / 2, gamma = rho s1 s2 i j / 4,
mu = r i / 2, nu = r j / 2.  Ring neighbours move to the right-hand side.
The interior matrix is assembled from these coefficients and solved directly
(sparse LU, one factorisation per (problem, dt)); the paper solves the same
system iteratively (Sec. 3.3), and any solver of it has this solution.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import Problem, bc, coords, payoff_grid

_LU_CACHE: dict = {}


def _index(M):
    n = M - 2
    return lambda i, j: (i - 1) * n + (j - 1)


def row_coefficients(p: Problem, dt: float, i: int, j: int) -> dict:
    """The nine entries of row (i, j) of (I - dt L_h), keyed by (di, dj)."""
    a = 0.5 * p.sigma1 * p.sigma1 * i * i
    b = 0.5 * p.sigma2 * p.sigma2 * j * j
    g = 0.25 * p.rho * p.sigma1 * p.sigma2 * i * j
    mu = 0.5 * p.r * i
    nu = 0.5 * p.r * j
    return {(0, 0): 1.0 + dt * (2.0 * a + 2.0 * b + p.r),
            (1, 0): -dt * (a + mu), (-1, 0): -dt * (a - mu),
            (0, 1): -dt * (b + nu), (0, -1): -dt * (b - nu),
            (1, 1): -dt * g, (-1, -1): -dt * g, (1, -1): dt * g, (-1, 1): dt * g}


def system(p: Problem, dt: float):
    """(A, R): A the interior matrix of (I - dt L_h) (CSC), R the map from the
    ring values (a full M x M grid, read on its ring only) to their
    contribution A_ring g, so that A u_int + R(g) is (I - dt L_h) u."""
    M = p.M
    n = M - 2
    idx = _index(M)
    rows, cols, vals = [], [], []
    ring_rows, ring_cols, ring_vals = [], [], []
    for i in range(1, M - 1):
        for j in range(1, M - 1):
            k = idx(i, j)
            for (di, dj), c in row_coefficients(p, dt, i, j).items():
                ii, jj = i + di, j + dj
                if 1 <= ii <= M - 2 and 1 <= jj <= M - 2:
                    rows.append(k)
                    cols.append(idx(ii, jj))
                    vals.append(c)
                else:
                    ring_rows.append(k)
                    ring_cols.append(ii * M + jj)
                    ring_vals.append(c)
    A = sp.csc_matrix((vals, (rows, cols)), shape=(n * n, n * n))
    R = sp.csr_matrix((ring_vals, (ring_rows, ring_cols)), shape=(n * n, M * M))
    return A, R


def _factor(p: Problem, dt: float):
    key = (p, float(dt))
    if key not in _LU_CACHE:
        A, R = system(p, dt)
        if len(_LU_CACHE) >= 2:   # a fine and a coarse step size of one problem at a time
            _LU_CACHE.pop(next(iter(_LU_CACHE)))
        _LU_CACHE[key] = (spla.splu(A), R)
    return _LU_CACHE[key]


def step_ring(p: Problem, dt: float, u: np.ndarray, ring1: np.ndarray) -> np.ndarray:
    """One implicit Euler step from the full grid u; ring1's ring holds the
    Dirichlet values at the new time.  Returns the new full grid."""
    M = p.M
    lu, R = _factor(p, dt)
    u = np.asarray(u, dtype=np.float64).reshape(M, M)
    ring1 = np.asarray(ring1, dtype=np.float64).reshape(M, M)
    rhs = u[1:-1, 1:-1].ravel() - R @ ring1.ravel()
    out = ring1.copy()
    out[1:-1, 1:-1] = lu.solve(rhs).reshape(M - 2, M - 2)
    return out


def ring_grid(p: Problem, tau: float) -> np.ndarray:
    """A full grid holding the boundary data g(., ., tau) on its ring (0 inside)."""
    M = p.M
    x = coords(p)
    g = np.zeros((M, M))
    for k in range(M):
        g[0, k] = bc(p, 0.0, x[k], tau)
        g[M - 1, k] = bc(p, x[M - 1], x[k], tau)
        g[k, 0] = bc(p, x[k], 0.0, tau)
        g[k, M - 1] = bc(p, x[k], x[M - 1], tau)
    return g


def fine(p: Problem, m: int, dt: float, tau0: float, u: np.ndarray, ring=None) -> np.ndarray:
    """F over one slice: m implicit steps of size dt from tau0.  ring(p, tau)
    gives the full grid of Dirichlet data (default: the oracle's boundary data)."""
    ring = ring or ring_grid
    for q in range(m):
        u = step_ring(p, dt, u, ring(p, tau0 + (q + 1) * dt))
    return u


def serial_fine(p: Problem, N: int, T: float, m: int, ring=None, init=None) -> np.ndarray:
    """u <- F(u) over slices n = 0..N-1 from the payoff (init(p), default the
    oracle's payoff grid); the state at tau = T."""
    dT = T / N
    u = (init or payoff_grid)(p)
    for n in range(N):
        u = fine(p, m, dT / m, n * dT, u, ring)
    return u
