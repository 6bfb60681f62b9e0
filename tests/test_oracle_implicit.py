"""Pins of the oracle's implicit-Euler fine propagator (Eq. (fd), Sec. 3.2).

* The assembled matrix against the explicit operator (pinned separately by
  the monomial eigenfunctions): A u_int + R(ring) = u - dt L_h u for any u.
* Exact discrete solutions: centred differences are exact on quadratic
  monomials, so with the monomial as initial value and the ring advanced by
  the same factor, implicit Euler gives exactly (1 - dt lambda)^{-m} x^a y^b.
* Convergence to Margrabe's closed form (first order in time, second in space)
  and unconditional stability at steps far above the explicit bound.
* Parareal (Eq. (parareal)) with the implicit F terminates exactly at K = N.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from oracle import implicit as im

C1 = dict(sigma1=0.3, sigma2=0.2, rho=0.5, r=0.05)


def prob(M, **kw):
    d = dict(C1)
    d.update(kw)
    return oracle.Problem(M=M, **d)


def test_matrix_equals_identity_minus_dt_operator():
    p = prob(17, rho=-0.6, r=0.08, sigma1=0.35)
    dt = 0.013
    A, R = im.system(p, dt)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((17, 17))
    lhs = A @ u[1:-1, 1:-1].ravel() + R @ u.ravel()
    rhs = (u - dt * oracle.apply_operator(p, u))[1:-1, 1:-1].ravel()
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


@pytest.mark.parametrize("rho", [0.5, -0.7])
@pytest.mark.parametrize("ab", [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1)])
def test_monomial_exact_discrete_solution(ab, rho):
    a, b = ab
    p = prob(33, rho=rho)
    x = oracle.coords(p)
    mono = np.outer(x ** a, x ** b)
    lam = cf.monomial_eigenvalue(a, b, p.sigma1, p.sigma2, p.rho, p.r)
    dt, m = 0.05, 20          # far above the explicit bound on 33^2 (about 0.0063)
    u = mono.copy()
    for q in range(m):
        u = im.step_ring(p, dt, u, mono * (1.0 - dt * lam) ** (-(q + 1)))
    expect = mono * (1.0 - dt * lam) ** (-m)
    assert np.abs(u - expect).max() <= 1e-12 * np.abs(expect).max()


def test_first_order_in_time_against_margrabe():
    """Exchange option with the exact ring: halving dt halves the time error at
    a fixed fine grid (the spatial error is small at 129^2 next to it)."""
    errs = []
    for m in (8, 16, 32):
        p = prob(129, payoff_kind=oracle.PAYOFF_EXCHANGE, bc_kind=oracle.BC_EXACT)
        u = im.serial_fine(p, 1, 1.0, m)
        k = 32   # node (1, 1)
        errs.append(u[k, k] - cf.margrabe(1.0, 1.0, 1.0, p.sigma1, p.sigma2, p.rho))
    assert abs(errs[0]) < 5e-3
    assert 1.6 <= errs[0] / errs[1] <= 2.4
    assert 1.6 <= errs[1] / errs[2] <= 2.6


def test_unconditionally_stable():
    """One step of 0.25 on 65^2 is 60 times the explicit bound; the basket
    call stays between 0 and the discounted ring maximum and is monotone."""
    p = prob(65)
    u = im.serial_fine(p, 1, 1.0, 4)
    assert np.isfinite(u).all()
    assert u.min() >= -1e-12
    assert u.max() <= 4.0 + 1e-12
    assert (np.diff(u, axis=0)[1:-1, 1:-1] >= -1e-12).all()


def test_parareal_with_implicit_fine_terminates_exactly():
    p = prob(17)
    pc = p.with_M(9)
    N, T, mF, mG = 4, 1.0, 6, 2
    dT = T / N
    Fn = lambda n, v: im.fine(p, mF, dT / mF, n * dT, v.reshape(17, 17))
    Gn = lambda n, v: oracle.coarse(p, pc, mG * 8, dT / (mG * 8), n * dT, v.reshape(17, 17))
    u0 = oracle.payoff_grid(p)
    ser = u0
    for n in range(N):
        ser = Fn(n, ser)
    U, K, _ = oracle.parareal_generic(u0, N, Fn, Gn, max_iters=N, tol=0.0)
    assert K == N
    assert np.array_equal(U[N].reshape(17, 17), ser)
