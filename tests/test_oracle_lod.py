"""Pins of the oracle's same-grid LOD coarse propagator (CPU only).

The step solves (I - dt Ly)(I - dt Lx) u+ = u + dt Lxy u with
Lx = alpha D_xx + mu D_x - r/2, Ly = beta D_yy + nu D_y - r/2, Lxy = gamma D_xy.
Quadratic monomials are eigenfunctions of all three difference operators, so
with the exact ring the step multiplies them by
(1 + dt lxy) / ((1 - dt lx)(1 - dt ly)) -- through both tridiagonal stages,
which pins every coefficient, sign and the intermediate boundary rows."""
import math

import numpy as np
import pytest

import oracle
from synthetic import plain_at_scale

C1 = dict(sigma1=0.3, sigma2=0.2, rho=0.5, r=0.05)


def eig(a, b, s1, s2, rho, r):
    lx = 0.5 * s1 * s1 * a * (a - 1) + r * a - 0.5 * r
    ly = 0.5 * s2 * s2 * b * (b - 1) + r * b - 0.5 * r
    lxy = rho * s1 * s2 * a * b
    return lx, ly, lxy


@pytest.mark.parametrize("rho", [0.5, -0.7])
@pytest.mark.parametrize("ab", [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1)])
def test_lod_monomial_exact(ab, rho):
    a, b = ab
    p = oracle.Problem(M=33, **dict(C1, rho=rho))
    x = oracle.coords(p)
    mono = np.outer(x ** a, x ** b)
    lx, ly, lxy = eig(a, b, p.sigma1, p.sigma2, p.rho, p.r)
    dt = 0.02   # far above the explicit limit: the implicit stages are what is tested
    fac = (1 + dt * lxy) / ((1 - dt * lx) * (1 - dt * ly))
    u = mono.copy()
    for q in range(5):
        u = oracle.lod_step_ring(p, dt, u, mono * fac ** (q + 1))
    assert np.abs(u - mono * fac ** 5).max() <= 1e-12 * max(1.0, np.abs(mono).max())


def test_lod_first_order_consistency():
    """LOD over one slice approaches the converged fine solution at first order in dt."""
    p = oracle.Problem(M=33, **C1)
    u0 = oracle.payoff_grid(p)
    dT = 0.125
    mref = oracle.steps_for(p, dT, 0.5) * 16
    ref = oracle.fine(p, mref, dT / mref, 0.0, u0)
    errs = [np.abs(oracle.lod(p, m, dT / m, 0.0, u0) - ref).max() for m in (8, 16, 32, 64)]
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert errs[-1] < 2e-4
    assert all(1.6 < q < 2.4 for q in ratios), (errs, ratios)


def test_lod_stable_far_above_explicit_limit():
    p = oracle.Problem(M=65, **C1)
    u0 = oracle.payoff_grid(p)
    dt = 50 * oracle.stable_dt(p)
    u = oracle.lod(p, 20, dt, 0.0, u0)
    assert np.isfinite(u).all() and np.abs(u).max() < 4.5


def test_parareal_with_lod_converges_fast():
    inst = plain_at_scale(1, M=65, n_slices=8)
    kw = dict(sigma1=inst.sigma1, sigma2=inst.sigma2, rho=inst.rho, r=inst.r, payoff_kind=0,
              w1=inst.w1, w2=inst.w2, strike=inst.strike)
    pf = oracle.Problem(M=65, **kw)
    dT = 1.0 / 8
    mF = oracle.steps_for(pf, dT, 0.9)
    ser = oracle.serial_fine(pf, 8, 1.0, mF)
    U, K, inc = oracle.parareal_bs(pf, pf, 8, 1.0, mF, 4, coarse_kind=oracle.G_LOD, tol=0.0,
                                   max_iters=8)
    assert K == 8 and np.array_equal(U, ser)          # finite termination, bitwise
    assert all(inc[k + 1] < 0.3 * inc[k] for k in range(4)), inc
    U4, K4, _ = oracle.parareal_bs(pf, pf, 8, 1.0, mF, 4, coarse_kind=oracle.G_LOD, tol=0.0,
                                   max_iters=4)
    assert np.abs(U4 - ser).max() / np.abs(ser).max() < 1e-6
