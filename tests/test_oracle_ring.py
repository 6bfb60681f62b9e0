"""Pins of the oracle's Dirichlet ring for the basket call (CPU only).

The ring value the oracle uses for the basket call is the forward intrinsic
value max(w1 S1 + w2 S2 - K e^{-r tau}, 0) (a reading of the "discounted
intrinsic value" boundary condition; the paper sets its ring from the closed
form of its option, Sec. 3.2).  These tests pin it against quantities the
mathematics fixes, computed here without the oracle's formula:

* the risk-neutral expectation of the basket call's payoff under the
  two-asset geometric Brownian motion of Eq. (bse), by two-dimensional
  Gauss-Hermite quadrature, at deep in-the-money ring nodes (where the call
  equals its forward to far below 1e-8) and deep out-of-the-money nodes;
* the same expectation without the max (the forward price), everywhere the
  max is inactive;
* the PDE itself: where the max is inactive the ring value solves
  Eq. (bse_change_variable), so d/dtau g = L_h g at every interior node.

A sign or placement error of e^{-r tau} (e^{+r tau}, discounting the whole
payoff, discounting with T instead of tau, dropping the strike's discount)
fails each of the first three groups.  The literal discounted payoff
(e^{-r tau} times the payoff, kept selectable) is pinned by values worked out
by hand from its definition and by its own time derivative.
"""
import math

import numpy as np
import pytest

import oracle

GH_POINTS = 200


def _gh():
    z, w = np.polynomial.hermite_e.hermegauss(GH_POINTS)
    w = w / math.sqrt(2.0 * math.pi)
    Z1, Z2 = np.meshgrid(z, z, indexing="ij")
    return Z1, Z2, np.outer(w, w)


def _terminal(x, y, tau, s1, s2, rho, r):
    """Asset prices at maturity under the risk-neutral two-asset GBM on the
    Gauss-Hermite nodes: correlated normals e1 = Z1, e2 = rho Z1 + sqrt(1-rho^2) Z2."""
    Z1, Z2, W = _gh()
    e2 = rho * Z1 + math.sqrt(1.0 - rho * rho) * Z2
    ST1 = x * np.exp((r - 0.5 * s1 * s1) * tau + s1 * math.sqrt(tau) * Z1)
    ST2 = y * np.exp((r - 0.5 * s2 * s2) * tau + s2 * math.sqrt(tau) * e2)
    return ST1, ST2, W


def basket_call_expectation(x, y, tau, s1, s2, rho, r, w1, w2, K):
    """e^{-r tau} E[max(w1 S1_T + w2 S2_T - K, 0)] and e^{-r tau} E[max(K - w.S_T, 0)]."""
    ST1, ST2, W = _terminal(x, y, tau, s1, s2, rho, r)
    basket = w1 * ST1 + w2 * ST2
    disc = math.exp(-r * tau)
    call = disc * float((np.maximum(basket - K, 0.0) * W).sum())
    put = disc * float((np.maximum(K - basket, 0.0) * W).sum())
    return call, put


def forward_expectation(x, y, tau, s1, s2, rho, r, w1, w2, K):
    """e^{-r tau} E[w1 S1_T + w2 S2_T - K] (smooth integrand: quadrature to rounding)."""
    ST1, ST2, W = _terminal(x, y, tau, s1, s2, rho, r)
    return math.exp(-r * tau) * float(((w1 * ST1 + w2 * ST2 - K) * W).sum())


PARAMS = [
    # sigma1, sigma2, rho, r, w1, w2, K
    (0.3, 0.2, 0.5, 0.05, 0.5, 0.5, 1.0),      # the 65^2 configuration's basket
    (0.15, 0.1, -0.6, 0.09, 0.7, 0.3, 0.8),
    (0.15, 0.2, 0.8, 0.02, 0.2, 0.8, 0.9),
]


def _problem(M, s1, s2, rho, r, w1, w2, K, bc_kind=oracle.BC_FORWARD_INTRINSIC):
    return oracle.Problem(M=M, sigma1=s1, sigma2=s2, rho=rho, r=r,
                          payoff_kind=oracle.PAYOFF_BASKET, w1=w1, w2=w2, strike=K,
                          bc_kind=bc_kind)


def _ring_nodes(p):
    x = oracle.coords(p)
    e = x[-1]
    nodes = []
    for t in x:
        nodes += [(0.0, t), (e, t), (t, 0.0), (t, e)]
    return nodes


@pytest.mark.parametrize("par", PARAMS)
@pytest.mark.parametrize("tau", [0.25, 1.0])
def test_basket_ring_matches_call_expectation_deep_itm(par, tau):
    """At ring nodes where the put part of the call's expectation is below
    1e-10 (deep in the money), the ring value equals the basket call's
    risk-neutral price to 1e-8."""
    s1, s2, rho, r, w1, w2, K = par
    p = _problem(33, *par)
    checked = 0
    for (x, y) in _ring_nodes(p):
        if w1 * x + w2 * y < 2.2 * K:
            continue
        call, put = basket_call_expectation(x, y, tau, s1, s2, rho, r, w1, w2, K)
        if put > 1e-10:
            continue
        checked += 1
        assert abs(oracle.bc(p, x, y, tau) - call) <= 1e-8, (x, y, tau)
    assert checked >= 8


@pytest.mark.parametrize("par", PARAMS)
def test_basket_ring_zero_deep_otm(par):
    """Where the basket is far below the strike the ring value is 0 and the
    call's price is below 1e-10."""
    s1, s2, rho, r, w1, w2, K = par
    p = _problem(33, *par)
    checked = 0
    for (x, y) in _ring_nodes(p):
        if w1 * x + w2 * y > 0.25 * K:
            continue
        call, _ = basket_call_expectation(x, y, 0.5, s1, s2, rho, r, w1, w2, K)
        assert call < 1e-10
        assert oracle.bc(p, x, y, 0.5) == 0.0
        checked += 1
    assert checked >= 2


@pytest.mark.parametrize("par", PARAMS)
@pytest.mark.parametrize("tau", [0.1, 0.6, 2.0])
def test_basket_ring_is_discounted_forward(par, tau):
    """Wherever the ring value is positive it equals the expected discounted
    basket minus strike (the forward price) to rounding; where it is 0 the
    forward is not positive."""
    s1, s2, rho, r, w1, w2, K = par
    p = _problem(65, *par)
    for (x, y) in _ring_nodes(p)[::3]:
        fwd = forward_expectation(x, y, tau, s1, s2, rho, r, w1, w2, K)
        g = oracle.bc(p, x, y, tau)
        if g > 0.0:
            assert abs(g - fwd) <= 1e-12 * max(1.0, abs(fwd)), (x, y)
        else:
            assert fwd <= 1e-12


@pytest.mark.parametrize("par", PARAMS)
def test_basket_ring_solves_the_pde_where_inactive(par):
    """g(., tau) on the whole grid: where w.S > K e^{-r tau} at a node and its
    eight neighbours, d/dtau g (central difference in tau) equals L_h g (the
    oracle's operator, pinned separately by the monomial eigenfunctions)."""
    s1, s2, rho, r, w1, w2, K = par
    p = _problem(33, *par)
    x = oracle.coords(p)
    tau, eps = 0.7, 1e-4

    def field(t):
        return np.array([[oracle.bc(p, a, b, t) for b in x] for a in x])

    g = field(tau)
    dg = (field(tau + eps) - field(tau - eps)) / (2.0 * eps)
    Lg = oracle.apply_operator(p, g)
    fwd = w1 * x[:, None] + w2 * x[None, :] - K * math.exp(-r * tau)
    inactive = fwd > 0.05
    ok = np.zeros_like(inactive)
    ok[1:-1, 1:-1] = np.all([inactive[1 + di:p.M - 1 + di, 1 + dj:p.M - 1 + dj]
                             for di in (-1, 0, 1) for dj in (-1, 0, 1)], axis=0)
    assert ok.sum() > 100
    # both equal r K e^{-r tau}; the tau difference is exact to O(eps^2) for an exponential
    want = r * K * math.exp(-r * tau)
    assert np.abs(Lg[ok] - want).max() <= 1e-12
    assert np.abs(dg[ok] - want).max() <= 1e-9 + 1e-8 * want


def test_discounted_payoff_ring_by_definition():
    """The literal reading, e^{-r tau} times the payoff, at values worked out by hand."""
    p = _problem(5, 0.3, 0.2, 0.5, 0.05, 0.5, 0.5, 1.0, bc_kind=oracle.BC_DISCOUNTED_PAYOFF)
    # basket (0.5, 0.5), K = 1 at (3, 1): payoff 1, tau = 1: e^{-0.05}
    assert abs(oracle.bc(p, 3.0, 1.0, 1.0) - 0.951229424500714) <= 1e-15
    # at (4, 4), tau = 2: payoff 3, discount e^{-0.1}
    assert abs(oracle.bc(p, 4.0, 4.0, 2.0) - 3.0 * 0.9048374180359595) <= 1e-15
    # out of the money: exactly 0 at any tau
    assert oracle.bc(p, 1.0, 0.5, 0.3) == 0.0
    # tau = 0: the payoff itself
    assert oracle.bc(p, 2.5, 0.5, 0.0) == 0.5
    pe = oracle.Problem(M=5, sigma1=0.3, sigma2=0.2, rho=0.5, r=0.05,
                        payoff_kind=oracle.PAYOFF_EXCHANGE,
                        bc_kind=oracle.BC_DISCOUNTED_PAYOFF)
    # exchange at (3, 1), tau = 2: payoff 2, discount e^{-0.1}
    assert abs(oracle.bc(pe, 3.0, 1.0, 2.0) - 1.809674836071919) <= 1e-15
    assert oracle.bc(pe, 1.0, 3.0, 2.0) == 0.0
    # d/dtau g = -r g (the discount runs in tau, not in T - tau)
    eps = 1e-5
    for (a, b, t) in [(3.0, 1.0, 0.4), (4.0, 2.0, 1.7)]:
        d = (oracle.bc(p, a, b, t + eps) - oracle.bc(p, a, b, t - eps)) / (2 * eps)
        assert abs(d + 0.05 * oracle.bc(p, a, b, t)) <= 1e-9
