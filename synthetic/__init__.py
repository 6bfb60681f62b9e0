"""Seeded synthetic workloads shared by the tests, the bench and the oracle.

This module holds only workload descriptions and random draws: which grid,
which model parameters, which payoff, how many slices.  It contains none of
the method's arithmetic (no stencil, no time stepping, no transfer), so the
HIP path and the oracle can both take their inputs from here without sharing
any computation.

The draws use ``numpy.random.default_rng(seed)`` (PCG64) in a fixed order:
sigma1, sigma2, rho, r, basket weights, strike, then (for the serving mix)
maturity, grid side and slice count.
"""
from __future__ import annotations

from dataclasses import asdict, dataclass, replace

import numpy as np

BASKET = 0
EXCHANGE = 1
CASH_OR_NOTHING = 2


@dataclass(frozen=True)
class Instance:
    """One pricing problem on an M x M grid over [0, s_max]^2."""
    M: int
    sigma1: float
    sigma2: float
    rho: float
    r: float
    T: float
    payoff: int = BASKET
    w1: float = 0.5
    w2: float = 0.5
    strike: float = 1.0
    s_max: float = 4.0
    n_slices: int = 8
    coarse_M: int = 33
    fine_steps_per_slice: int = 0      # 0: planned from cfl
    coarse_steps_per_slice: int = 0    # 0: planned from cfl
    cfl: float = 0.9
    fp32: bool = False
    tol: float = 1e-8
    tol_relative: bool = False
    implicit: bool = False             # implicit-Euler fine propagator (fine_steps_per_slice > 0)
    krylov_tol: float = 0.0            # 0: the library's default
    strike2: float = 0.0               # cash-or-nothing: second strike (strike is the first)
    cash: float = 0.0                  # cash-or-nothing: cash amount

    def replace(self, **kw) -> "Instance":
        return replace(self, **kw)

    def as_dict(self) -> dict:
        return asdict(self)


def plain_fp64(payoff: int = BASKET) -> Instance:
    """65 x 65 grid on [0,4]^2, s1=0.3, s2=0.2, rho=0.5, r=0.05, T=1; basket
    (0.5, 0.5) with K=1 or the exchange option; F = 1024 explicit steps in
    total (128 per slice over 8 slices), G = 64 steps per slice on 33 x 33;
    stop when the max increment is below 1e-8.  Everything in FP64."""
    return Instance(M=65, sigma1=0.3, sigma2=0.2, rho=0.5, r=0.05, T=1.0, payoff=payoff,
                    w1=0.5, w2=0.5, strike=1.0, n_slices=8, coarse_M=33,
                    fine_steps_per_slice=128, coarse_steps_per_slice=64, fp32=False,
                    tol=1e-8, tol_relative=False)


def draw_params(rng: np.random.Generator) -> dict:
    """sigma1, sigma2 ~ U[0.1, 0.5]; rho ~ U[-0.8, 0.8]; r ~ U[0, 0.1];
    basket weights ~ Dirichlet(1, 1); strike ~ U[0.5, 1.5]."""
    s1 = float(rng.uniform(0.1, 0.5))
    s2 = float(rng.uniform(0.1, 0.5))
    rho = float(rng.uniform(-0.8, 0.8))
    r = float(rng.uniform(0.0, 0.1))
    w = rng.dirichlet([1.0, 1.0])
    K = float(rng.uniform(0.5, 1.5))
    return dict(sigma1=s1, sigma2=s2, rho=rho, r=r, w1=float(w[0]), w2=float(w[1]), strike=K)


def plain_at_scale(seed: int, M: int = 513, n_slices: int = 64, coarse_M: int = 129) -> Instance:
    """513 x 513 FP32 fine grid with FP64 correction, seed-drawn parameters,
    T = 1, N = 64 slices, numerical coarse grid 129 x 129, dt at 0.9 of the
    explicit stability limit on both grids; stop when the max increment is
    below 1e-7 of the solution's max norm."""
    rng = np.random.default_rng(seed)
    return Instance(M=M, T=1.0, payoff=BASKET, n_slices=n_slices, coarse_M=coarse_M, cfl=0.9,
                    fp32=True, tol=1e-7, tol_relative=True, **draw_params(rng))


def largest_single() -> Instance:
    """2049 x 2049 FP32 grid, N = 256 slices, basket (0.6, 0.4) with K = 1,
    s1=0.35, s2=0.25, rho=0.3, r=0.03, T=2, numerical coarse grid 257 x 257."""
    return Instance(M=2049, sigma1=0.35, sigma2=0.25, rho=0.3, r=0.03, T=2.0, payoff=BASKET,
                    w1=0.6, w2=0.4, strike=1.0, n_slices=256, coarse_M=257, cfl=0.9, fp32=True,
                    tol=1e-7, tol_relative=True)


def paper_benchmark(n_slices: int = 10, fine_steps_per_slice: int = 3, spacing: float = 1.0,
                    **kw) -> Instance:
    """The paper's test problem (Sec. 3.2): two-asset cash-or-nothing option on
    [0, 300]^2 with node spacing 1 (301 x 301), strikes 100 and 100, r = 1,
    sigma1 = sigma2 = 0.3, rho = 0.5, T = 1, closed-form ring; implicit Euler
    with coarse step 0.1 (one step per slice over 10 slices) and the fine step a
    third of it.  The cash amount is not printed; c = 1.  `spacing` 0.5 or 0.25
    gives the refined grids of Sec. 4.4 (601^2, 1201^2)."""
    M = int(round(300.0 / spacing)) + 1
    d = dict(M=M, sigma1=0.3, sigma2=0.3, rho=0.5, r=1.0, T=1.0, payoff=CASH_OR_NOTHING, w1=0.0,
             w2=0.0, strike=100.0, strike2=100.0, cash=1.0, s_max=300.0, n_slices=n_slices,
             coarse_M=M, fine_steps_per_slice=fine_steps_per_slice, coarse_steps_per_slice=1,
             fp32=False, tol=0.0, tol_relative=False, implicit=True, krylov_tol=1e-12)
    d.update(kw)
    return Instance(**d)


@dataclass(frozen=True)
class Instance3:
    """One three-asset pricing problem (Eq. (bse_general), n = 3) on an M^3 grid
    over [0, s_max]^3, basket call max(w . S - K, 0); rho = (rho12, rho13, rho23)."""
    M: int
    coarse_M: int
    sigma: tuple
    rho: tuple
    r: float
    T: float
    w: tuple
    strike: float
    n_slices: int = 8
    s_max: float = 4.0
    tol: float = 0.0
    max_iters: int = 0
    fine_steps: int = 0
    coarse_steps: int = 0
    cfl: float = 0.9

    def replace(self, **kw) -> "Instance3":
        return replace(self, **kw)


def three_asset(seed: int, M: int = 65, coarse_M: int = 17, n_slices: int = 16,
                T: float = 1.0) -> Instance3:
    """sigma_d ~ U[0.1, 0.5]; (rho12, rho13, rho23) ~ U[-0.5, 0.5] each, drawn
    again until the correlation matrix is positive definite; r ~ U[0, 0.1];
    weights ~ Dirichlet(1, 1, 1); K ~ U[0.5, 1.5]."""
    rng = np.random.default_rng(seed)
    sigma = tuple(float(x) for x in rng.uniform(0.1, 0.5, size=3))
    while True:
        rho = tuple(float(x) for x in rng.uniform(-0.5, 0.5, size=3))
        a, b, c = rho
        if 1.0 - a * a - b * b - c * c + 2.0 * a * b * c > 0.0:
            break
    r = float(rng.uniform(0.0, 0.1))
    w = tuple(float(x) for x in rng.dirichlet([1.0, 1.0, 1.0]))
    K = float(rng.uniform(0.5, 1.5))
    return Instance3(M=M, coarse_M=coarse_M, sigma=sigma, rho=rho, r=r, T=T, w=w, strike=K,
                     n_slices=n_slices)


SERVE_SIDES = (129, 257, 513, 1025)
SERVE_SLICES = (16, 32, 64)


def serving_requests(rate: float, count: int, seed: int, sides=SERVE_SIDES):
    """Poisson arrivals at `rate` requests/s: returns (arrival_times, instances).

    Grid side uniform over `sides` (log-uniform over 129..1025, which are
    equally spaced in log), N uniform over {16, 32, 64}, model parameters and
    payoff as in the seeded at-scale draw, T ~ U[0.25, 2]; numerical coarse
    grid (M-1)/4 + 1."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for _ in range(count):
        p = draw_params(rng)
        T = float(rng.uniform(0.25, 2.0))
        M = int(sides[int(rng.integers(len(sides)))])
        N = int(SERVE_SLICES[int(rng.integers(len(SERVE_SLICES)))])
        out.append(Instance(M=M, T=T, payoff=BASKET, n_slices=N, coarse_M=(M - 1) // 4 + 1,
                            cfl=0.9, fp32=True, tol=1e-7, tol_relative=True, **p))
    return t, out


FNO_GRID = 64


def fno_batch(seed: int, batch: int):
    """Random inputs of the 64 x 64 neural operator: a plane w per sample (a few
    random low sine modes plus small noise, zero on the ring) and the model
    parameters (sigma1, sigma2, rho, r) drawn as in the at-scale problem.
    Returns float32 arrays w (batch, 64, 64) and meta (batch, 4)."""
    rng = np.random.default_rng(seed)
    t = np.linspace(0.0, 1.0, FNO_GRID)
    w = np.zeros((batch, FNO_GRID, FNO_GRID))
    meta = np.zeros((batch, 4))
    for b in range(batch):
        p = draw_params(rng)
        meta[b] = (p["sigma1"], p["sigma2"], p["rho"], p["r"])
        for _ in range(4):
            kx, ky = rng.integers(1, 9, size=2)
            w[b] += rng.normal(0.0, 0.1) * np.outer(np.sin(np.pi * kx * t), np.sin(np.pi * ky * t))
        w[b, 1:-1, 1:-1] += rng.normal(0.0, 0.01, size=(FNO_GRID - 2, FNO_GRID - 2))
        w[b, [0, -1], :] = 0.0
        w[b, :, [0, -1]] = 0.0
    return w.astype(np.float32), meta.astype(np.float32)


def fno_pairs(seed: int, batch: int):
    """Random training pairs [w_in, B1, V_in, V_tgt] (batch, 4, 64, 64) float32 with
    the magnitudes of option values on [0, 4]^2 (a smooth ramp plus the random
    planes of fno_batch), and their meta (batch, 4)."""
    w, meta = fno_batch(seed, batch)
    rng = np.random.default_rng(seed + 7919)
    x = np.linspace(0.0, 4.0, FNO_GRID)
    ramp = 0.5 * (x[:, None] + x[None, :])
    pairs = np.zeros((batch, 4, FNO_GRID, FNO_GRID))
    for b in range(batch):
        a0 = rng.uniform(0.9, 1.1)
        pairs[b, 0] = w[b]
        pairs[b, 1] = a0 * ramp
        pairs[b, 2] = 0.99 * a0 * ramp + w[b]
        pairs[b, 3] = a0 * ramp + w[b] + rng.normal(0.0, 1e-3, size=(FNO_GRID, FNO_GRID))
    return pairs.astype(np.float32), meta
