"""The paper's benchmark problem: the two-asset cash-or-nothing option of
Sec. 3.2 (TEST INFRASTRUCTURE ONLY; only tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py may import it).

* Payoff at maturity: c if S1 >= K1 and S2 >= K2, else 0.
* Closed form, Eq. (solution): c e^{-r tau} B(d1, d2; rho) with
  d_i = (ln(S_i / K_i) + (r - sigma_i^2 / 2) tau) / (sigma_i sqrt(tau)) and B the
  bivariate standard normal CDF; the paper also uses it as the Dirichlet data.
* B evaluated through Owen's T function (scipy.special.owens_t):
      B(h, k; rho) = [Phi(h) + Phi(k)] / 2 - T(h, a_h) - T(k, a_k) - delta,
      a_h = (k - rho h) / (h sqrt(1 - rho^2)), a_k = (h - rho k) / (k sqrt(1 - rho^2)),
      delta = 0 if h k > 0 or (h k = 0 and h + k >= 0), else 1/2
  (Owen, 1956), a different route from the quadrature of the GPU path.
* The paper's configuration: [0, 300]^2 with spacing 1 (301 x 301 nodes),
  K1 = K2 = 100, r = 1, sigma1 = sigma2 = 0.3, rho = 0.5, T = 1; the cash
  amount is not printed and is taken as c = 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import ndtr, owens_t


@dataclass(frozen=True)
class CashProblem:
    M: int = 301
    s_max: float = 300.0
    sigma1: float = 0.3
    sigma2: float = 0.3
    rho: float = 0.5
    r: float = 1.0
    K1: float = 100.0
    K2: float = 100.0
    cash: float = 1.0

    @property
    def h(self) -> float:
        return self.s_max / (self.M - 1)


def paper_problem() -> CashProblem:
    return CashProblem()


def bvn_cdf(h, k, rho):
    """P(X <= h, Y <= k) for standard normals with correlation rho (arrays broadcast)."""
    h, k = np.broadcast_arrays(np.asarray(h, dtype=np.float64), np.asarray(k, dtype=np.float64))
    out = np.zeros(h.shape)
    sq = np.sqrt(1.0 - rho * rho)
    fin = np.isfinite(h) & np.isfinite(k)
    hp, kp = h == np.inf, k == np.inf
    out[hp & kp] = 1.0
    out[hp & np.isfinite(k)] = ndtr(k[hp & np.isfinite(k)])
    out[kp & np.isfinite(h)] = ndtr(h[kp & np.isfinite(h)])
    zz = fin & (h == 0.0) & (k == 0.0)
    out[zz] = 0.25 + np.arcsin(rho) / (2.0 * np.pi)
    g = fin & ~zz
    hg, kg = h[g], k[g]
    with np.errstate(divide="ignore", invalid="ignore"):
        ah = np.where(hg != 0.0, (kg - rho * hg) / (hg * sq), np.sign(kg) * np.inf)
        ak = np.where(kg != 0.0, (hg - rho * kg) / (kg * sq), np.sign(hg) * np.inf)
    delta = np.where((hg * kg > 0.0) | ((hg * kg == 0.0) & (hg + kg >= 0.0)), 0.0, 0.5)
    out[g] = 0.5 * (ndtr(hg) + ndtr(kg)) - owens_t(hg, ah) - owens_t(kg, ak) - delta
    return out


def payoff(p: CashProblem, x, y):
    return np.where((np.asarray(x) >= p.K1) & (np.asarray(y) >= p.K2), p.cash, 0.0)


def closed_form(p: CashProblem, x, y, tau):
    """Eq. (solution): c e^{-r tau} B(d1, d2; rho); the payoff at tau = 0."""
    x, y = np.broadcast_arrays(np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64))
    if tau <= 0.0:
        return payoff(p, x, y)
    st = np.sqrt(tau)
    with np.errstate(divide="ignore"):
        d1 = (np.log(x / p.K1) + (p.r - 0.5 * p.sigma1 ** 2) * tau) / (p.sigma1 * st)
        d2 = (np.log(y / p.K2) + (p.r - 0.5 * p.sigma2 ** 2) * tau) / (p.sigma2 * st)
    return p.cash * np.exp(-p.r * tau) * bvn_cdf(d1, d2, p.rho)


def coords(p: CashProblem) -> np.ndarray:
    return np.arange(p.M, dtype=np.float64) * p.h


def exact_grid(p: CashProblem, tau: float) -> np.ndarray:
    x = coords(p)
    return closed_form(p, x[:, None], x[None, :], tau)


def payoff_grid(p: CashProblem) -> np.ndarray:
    x = coords(p)
    return payoff(p, x[:, None], x[None, :]).astype(np.float64)


def ring_grid(p: CashProblem, tau: float) -> np.ndarray:
    """A full grid with the closed form on its ring (0 inside)."""
    g = exact_grid(p, tau)
    g[1:-1, 1:-1] = 0.0
    return g


def rel_l2(u, ref) -> float:
    return float(np.linalg.norm(u - ref) / np.linalg.norm(ref))
