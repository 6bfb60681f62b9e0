"""Closed-form option prices used to pin the oracle (TEST INFRASTRUCTURE ONLY).

Written independently of ``bs2d.c``: pure Python ``math``.

* Margrabe's exchange-option price: the exact solution of
  Eq. (bse_change_variable) (Sec. 3.2) for the payoff max(S1 - S2, 0).
* The one-asset Black-Scholes call: the exact solution of the same PDE for a
  basket with weights (1, 0), which does not depend on S2, sigma2 or rho.
* The quadratic-monomial eigenvalues of the operator of Eq. (fd): centred
  differences are exact on polynomials of degree <= 2, so
  L_h(x^a y^b) = lambda_ab x^a y^b with
  lambda_ab = 1/2 s1^2 a(a-1) + 1/2 s2^2 b(b-1) + rho s1 s2 a b + r (a + b) - r.
"""
from __future__ import annotations

import math


def ncdf(z: float) -> float:
    return 0.5 * math.erfc(-z / math.sqrt(2.0))


def margrabe(s1_price: float, s2_price: float, tau: float, sigma1: float, sigma2: float,
             rho: float) -> float:
    """Price of max(S1 - S2, 0) at time-to-maturity tau (r cancels)."""
    if tau <= 0.0:
        return max(s1_price - s2_price, 0.0)
    if s1_price <= 0.0:
        return 0.0
    if s2_price <= 0.0:
        return s1_price
    vol = math.sqrt(sigma1 ** 2 + sigma2 ** 2 - 2.0 * rho * sigma1 * sigma2)
    sd = vol * math.sqrt(tau)
    d1 = (math.log(s1_price / s2_price) + 0.5 * sd * sd) / sd
    return s1_price * ncdf(d1) - s2_price * ncdf(d1 - sd)


def bs_call(S: float, K: float, r: float, sigma: float, tau: float) -> float:
    """One-asset European call."""
    if tau <= 0.0:
        return max(S - K, 0.0)
    if S <= 0.0:
        return 0.0
    sd = sigma * math.sqrt(tau)
    d1 = (math.log(S / K) + (r + 0.5 * sigma * sigma) * tau) / sd
    return S * ncdf(d1) - K * math.exp(-r * tau) * ncdf(d1 - sd)


def monomial_eigenvalue(a: int, b: int, sigma1: float, sigma2: float, rho: float, r: float) -> float:
    """lambda_ab for x^a y^b, a + b <= 2 (exact for both L and L_h)."""
    return (0.5 * sigma1 ** 2 * a * (a - 1) + 0.5 * sigma2 ** 2 * b * (b - 1)
            + rho * sigma1 * sigma2 * a * b + r * (a + b) - r)


def scalar_parareal(f: float, g: float, u0: float, k: int, n: int) -> float:
    """U^k_n for Parareal with F = f*I, G = g*I: sum_{j<=min(k,n)} C(n,j) (f-g)^j g^(n-j) u0.

    Follows by induction from Eq. (parareal) with U^0_n = g^n u0."""
    return sum(math.comb(n, j) * (f - g) ** j * g ** (n - j) for j in range(min(k, n) + 1)) * u0
