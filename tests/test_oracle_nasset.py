"""Pins of the three-asset oracle (Eq. (bse_general), Sec. 3.2) against what
the mathematics fixes, independent of the oracle's own formulas:

* monomials x^a y^b z^c with a, b, c <= 2 are exact eigenfunctions of the
  centred 19-point operator, with the eigenvalue of the continuous operator
  (distinct sigmas and correlations, so a swapped pair or a dropped term fails);
* explicit Euler then multiplies them by exactly (1 + dt lambda) per step;
* with no correlation to the third asset, a payoff that ignores it and faces
  that carry the two-asset solution, every plane is the two-asset oracle's
  solution (the C oracle, written separately);
* permuting the assets permutes the solution;
* the stability bound equals a brute-force Gershgorin bound of the assembled
  matrix;
* injection after trilinear prolongation returns the coarse values bitwise,
  and prolongation reproduces trilinear functions;
* Parareal over these propagators terminates at serial F after N iterations
  and in one iteration when G = F.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import nasset as na

P = na.Problem3(M=9, sigma=(0.3, 0.2, 0.45), rho=(0.5, -0.3, 0.2), r=0.07,
                w=(0.5, 0.3, 0.2), strike=1.0)


def monomial(p, e):
    X = np.meshgrid(*(na.coords(p),) * 3, indexing="ij")
    return X[0] ** e[0] * X[1] ** e[1] * X[2] ** e[2]


def eigenvalue(p, e):
    s, (r12, r13, r23) = p.sigma, p.rho
    lam = sum(0.5 * s[d] ** 2 * e[d] * (e[d] - 1) for d in range(3))
    lam += r12 * s[0] * s[1] * e[0] * e[1] + r13 * s[0] * s[2] * e[0] * e[2]
    lam += r23 * s[1] * s[2] * e[1] * e[2]
    return lam + p.r * sum(e) - p.r


@pytest.mark.parametrize("e", list(itertools.product(range(3), repeat=3)))
def test_monomials_are_eigenfunctions(e):
    u = monomial(P, e)
    got = na.apply_operator(P, u)
    want = eigenvalue(P, e) * u[1:-1, 1:-1, 1:-1]
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(u).max())


def test_euler_multiplies_a_monomial():
    e = (2, 1, 2)
    lam = eigenvalue(P, e)
    u0 = monomial(P, e)
    dt, m = 1e-3, 7
    faces = lambda p, tau: u0 * (1.0 + dt * lam) ** round(tau / dt)
    u = na.fine(P, m, dt, 0.0, u0, faces=faces)
    assert np.allclose(u, u0 * (1.0 + dt * lam) ** m, rtol=1e-12, atol=1e-13)


def test_reduces_to_the_two_asset_scheme():
    p3 = na.Problem3(M=17, sigma=(0.35, 0.25, 0.4), rho=(0.4, 0.0, 0.0), r=0.05,
                     w=(0.6, 0.4, 0.0), strike=1.0)
    p2 = oracle.Problem(M=17, sigma1=0.35, sigma2=0.25, rho=0.4, r=0.05, w1=0.6, w2=0.4,
                        strike=1.0)
    dt = 0.9 * na.stable_dt(p3)
    # the 2-D solution after every step; the 3-D faces carry it (constant along
    # x3), so that the x3 = 0 and x3 = s_max planes hold what the 2-D scheme
    # computes there
    hist = [oracle.payoff_grid(p2)]
    for q in range(20):
        hist.append(oracle.fine(p2, 1, dt, q * dt, hist[-1]))
    faces = lambda p, tau: np.repeat(hist[round(tau / dt)][:, :, None], 17, axis=2)
    u3 = na.fine(p3, 20, dt, 0.0, na.payoff_grid(p3), faces=faces)
    for k in range(17):
        assert np.allclose(u3[:, :, k], hist[-1], rtol=0, atol=1e-13), k
    assert np.abs(hist[-1] - hist[0]).max() > 1e-3   # the solution did move


def test_permuting_assets_permutes_the_solution():
    perm = (2, 0, 1)   # new axis d is old axis perm[d]
    pair = {(0, 1): 0, (0, 2): 1, (1, 2): 2}
    rho = tuple(P.rho[pair[tuple(sorted((perm[d], perm[e])))]] for d, e in na.PAIRS)
    q = na.Problem3(M=P.M, sigma=tuple(P.sigma[perm[d]] for d in range(3)), rho=rho, r=P.r,
                    w=tuple(P.w[perm[d]] for d in range(3)), strike=P.strike)
    dt = 0.9 * na.stable_dt(P)
    u = na.fine(P, 15, dt, 0.0, na.payoff_grid(P))
    v = na.fine(q, 15, dt, 0.0, na.payoff_grid(q))
    assert np.allclose(v, np.transpose(u, perm), rtol=0, atol=1e-14)


def test_stable_dt_is_the_gershgorin_bound_of_the_matrix():
    """Rows of L_h assembled column by column over every node (the face nodes
    included: their couplings count in the row sums of explicit Euler)."""
    p = P.with_M(6)
    n, M = p.M - 2, p.M
    A = np.zeros((n ** 3, M ** 3))
    for col in range(M ** 3):
        u = np.zeros((M,) * 3)
        u.flat[col] = 1.0
        A[:, col] = na.apply_operator(p, u).ravel()
    inner = np.zeros((M,) * 3, dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    diag = A[:, np.flatnonzero(inner)].diagonal()
    rows = np.abs(diag) + (np.abs(A).sum(axis=1) - np.abs(diag))
    assert math.isclose(na.stable_dt(p), 2.0 / rows.max(), rel_tol=1e-14)


def test_transfers():
    rng = np.random.default_rng(3)
    c = rng.standard_normal((5, 5, 5))
    assert np.array_equal(na.restrict(na.prolong(c, 4), 4), c)
    x = np.linspace(0.0, 1.0, 5)
    X = np.meshgrid(x, x, x, indexing="ij")
    f = lambda a, b, d: 1.0 + 2.0 * a - b + 0.5 * d + 3.0 * a * b * d - a * d
    xf = np.linspace(0.0, 1.0, 17)
    XF = np.meshgrid(xf, xf, xf, indexing="ij")
    assert np.allclose(na.prolong(f(*X), 4), f(*XF), atol=1e-13)


@pytest.mark.parametrize("same", [False, True])
def test_parareal_over_three_assets(same):
    """N = 4 slices of 0.05 on 9^3; G on 5^3 (or G = F): K = N gives serial F
    bitwise, and G = F converges in one iteration."""
    p = P
    N, T = 4, 0.2
    dT = T / N
    mF = na.steps_for(p, dT)
    mG = na.steps_for(p.with_M(5), dT)
    Fn = lambda n, v: na.fine(p, mF, dT / mF, n * dT, v.reshape((p.M,) * 3))
    if same:
        Gn = Fn
    else:
        Gn = lambda n, v: na.coarse(p, 5, mG, dT / mG, n * dT, v.reshape((p.M,) * 3))
    U, K, _ = oracle.parareal_generic(na.payoff_grid(p), N, Fn, Gn,
                                      max_iters=1 if same else N, tol=0.0)
    ser = na.serial_fine(p, N, T, mF)
    assert np.array_equal(U[-1].reshape(ser.shape), ser)
    assert K == (1 if same else N)
