"""Pins of the oracle's cash-or-nothing module (the paper's benchmark, Sec. 3.2).

* The bivariate normal CDF (Owen's T route) against its definition: numerical
  integration of the bivariate density, the product form at rho = 0, the
  closed value at the origin, a reflection identity and the limits.
* The closed form of Eq. (solution) against the PDE (finite differences) and
  its limits (payoff at tau -> 0, zero on the axes, the one-asset digital as the
  other asset grows).
* The implicit-Euler oracle on this problem converges to the closed form at
  first order in the time step.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import ndtr

from oracle import cash
from oracle import implicit as im


def density(x, y, rho):
    q = (x * x - 2 * rho * x * y + y * y) / (2 * (1 - rho * rho))
    return math.exp(-q) / (2 * math.pi * math.sqrt(1 - rho * rho))


@pytest.mark.parametrize("h,k,rho", [(0.3, -0.7, 0.5), (-1.2, 0.4, -0.6), (1.5, 2.0, 0.85),
                                     (-0.2, -0.3, 0.0), (0.0, 1.1, -0.9)])
def test_bvn_against_density_integral(h, k, rho):
    val, _ = integrate.dblquad(lambda y, x: density(x, y, rho), -12.0, h, -12.0, k,
                               epsabs=1e-13, epsrel=1e-12)
    assert abs(cash.bvn_cdf(h, k, rho) - val) < 1e-10


def test_bvn_identities():
    rng = np.random.default_rng(4)
    h, k = rng.normal(size=50) * 1.5, rng.normal(size=50) * 1.5
    for rho in (-0.8, -0.3, 0.4, 0.92):
        b = cash.bvn_cdf(h, k, rho)
        assert np.allclose(b, cash.bvn_cdf(k, h, rho), atol=1e-14, rtol=0)         # symmetry
        assert np.allclose(b + cash.bvn_cdf(h, -k, -rho), ndtr(h), atol=1e-13, rtol=0)   # reflection
    assert np.allclose(cash.bvn_cdf(h, k, 0.0), ndtr(h) * ndtr(k), atol=1e-15, rtol=0)
    for rho in (-0.7, 0.2, 0.5):
        assert abs(cash.bvn_cdf(0.0, 0.0, rho) - (0.25 + math.asin(rho) / (2 * math.pi))) < 1e-15
    assert cash.bvn_cdf(-np.inf, 0.3, 0.5) == 0.0
    assert abs(cash.bvn_cdf(np.inf, 0.3, 0.5) - ndtr(0.3)) < 1e-16


def test_closed_form_solves_the_pde():
    p = cash.paper_problem()
    f = lambda a, b, t: float(cash.closed_form(p, a, b, t))
    for (x, y, t) in [(110.0, 95.0, 0.7), (80.0, 130.0, 0.3), (150.0, 150.0, 1.0)]:
        e, h = 1e-4, 0.02
        ut = (f(x, y, t + e) - f(x, y, t - e)) / (2 * e)
        uxx = (f(x + h, y, t) - 2 * f(x, y, t) + f(x - h, y, t)) / h ** 2
        uyy = (f(x, y + h, t) - 2 * f(x, y, t) + f(x, y - h, t)) / h ** 2
        uxy = (f(x + h, y + h, t) - f(x + h, y - h, t) - f(x - h, y + h, t) + f(x - h, y - h, t)) / (4 * h * h)
        ux = (f(x + h, y, t) - f(x - h, y, t)) / (2 * h)
        uy = (f(x, y + h, t) - f(x, y - h, t)) / (2 * h)
        L = (0.5 * p.sigma1 ** 2 * x * x * uxx + 0.5 * p.sigma2 ** 2 * y * y * uyy
             + p.rho * p.sigma1 * p.sigma2 * x * y * uxy + p.r * x * ux + p.r * y * uy - p.r * f(x, y, t))
        assert abs(ut - L) <= 1e-5 * max(abs(ut), 1e-3), (x, y, t, ut, L)


def test_closed_form_limits():
    p = cash.paper_problem()
    # tau -> 0: the payoff, away from the strike lines
    assert abs(float(cash.closed_form(p, 120.0, 130.0, 1e-8)) - math.exp(-p.r * 1e-8)) < 1e-12
    assert float(cash.closed_form(p, 80.0, 130.0, 1e-8)) < 1e-12
    # either asset at 0: worth nothing
    assert float(cash.closed_form(p, 0.0, 150.0, 0.5)) == 0.0
    # the second asset far in the money: the one-asset digital c e^{-r tau} N(d1)
    tau, x = 0.6, 104.0
    d1 = (math.log(x / p.K1) + (p.r - 0.5 * p.sigma1 ** 2) * tau) / (p.sigma1 * math.sqrt(tau))
    assert abs(float(cash.closed_form(p, x, 1e6, tau)) - p.cash * math.exp(-p.r * tau) * ndtr(d1)) < 1e-14


def test_implicit_oracle_first_order_to_closed_form():
    p = cash.CashProblem(M=121, s_max=300.0)   # spacing 2.5
    ex = cash.exact_grid(p, 1.0)
    errs = []
    for m in (4, 8, 16):
        u = im.serial_fine(p, 5, 1.0, m, ring=cash.ring_grid, init=cash.payoff_grid)
        errs.append(cash.rel_l2(u, ex))
    assert errs[0] > errs[1] > errs[2]
    assert 1.5 <= errs[0] / errs[1] <= 2.5 and 1.4 <= errs[1] / errs[2] <= 2.5
