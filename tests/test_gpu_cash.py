"""The paper's benchmark problem on the GPU (Sec. 3.2): the two-asset
cash-or-nothing option on [0, 300]^2 with the closed form of Eq. (solution) as
Dirichlet data, implicit-Euler F and the implicit-Euler numerical G on the same
grid, against the oracle (bivariate normal CDF through Owen's T, direct sparse
solves).
"""
import numpy as np
import pytest

import oracle
from oracle import cash
from oracle import implicit as im
from helpers import abs_max, say
from synthetic import paper_benchmark

pytestmark = pytest.mark.gpu
FP64_TOL = 1e-10


@pytest.fixture(scope="module")
def pr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2404_02521_amd as pr_
    return pr_


def host(t):
    return t.detach().cpu().numpy()


def cprob(inst):
    return cash.CashProblem(M=inst.M, s_max=inst.s_max, sigma1=inst.sigma1, sigma2=inst.sigma2,
                            rho=inst.rho, r=inst.r, K1=inst.strike, K2=inst.strike2,
                            cash=inst.cash)


@pytest.mark.parametrize("rho,T", [(0.5, 1.0), (-0.9, 0.4), (0.0, 2.0), (0.92, 0.05), (-0.3, 3.0)])
def test_device_bivariate_cdf_on_the_ring(pr, rho, T):
    """The ring of the returned grid is the closed form at tau = T evaluated on
    the device (Plackett's identity, 20-point Gauss-Legendre): against the
    oracle's Owen's-T evaluation at every ring node."""
    inst = paper_benchmark(spacing=5.0, rho=rho, T=T, n_slices=1, fine_steps_per_slice=1)
    say("device BVN ring", rho, T)
    s = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT, coarse_kind=pr.PR_G_IMPLICIT)
    v = host(s.serial_fine().value)
    ex = cash.exact_grid(cprob(inst), T)
    ring = np.ones_like(ex, dtype=bool)
    ring[1:-1, 1:-1] = False
    assert np.abs(v[ring] - ex[ring]).max() <= 1e-14
    s.close()


def test_serial_fine_reduced_grid_vs_oracle(pr):
    """Spacing 5 (61^2), 10 slices x 3 implicit steps: against the oracle."""
    inst = paper_benchmark(spacing=5.0, krylov_tol=1e-13)
    say("cash serial F 61^2")
    s = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT, coarse_kind=pr.PR_G_IMPLICIT)
    got = host(s.serial_fine().value)
    ref = im.serial_fine(cprob(inst), 10, 1.0, 3, ring=cash.ring_grid, init=cash.payoff_grid)
    assert abs_max(got, ref) <= FP64_TOL
    s.close()


def test_paper_grid_serial_fine_and_coarse_vs_oracle(pr):
    """The paper's 301^2 grid: serial F (30 steps of 1/30) and the numerical G
    alone (10 steps of 0.1) against the oracle, and their relative l2 errors
    against the closed form (the quantities Sec. 4.1 prints for its own runs)."""
    inst = paper_benchmark(krylov_tol=1e-13)
    p = cprob(inst)
    say("cash serial F and G 301^2")
    s = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT, coarse_kind=pr.PR_G_IMPLICIT)
    sf = s.serial_fine()
    f = host(sf.value)
    print("Krylov iterations per fine step", sf.stats["krylov_iters"] / 30,
          "max", sf.stats["krylov_max_step"])
    assert sf.stats["krylov_unconverged"] == 0
    ref_f = im.serial_fine(p, 10, 1.0, 3, ring=cash.ring_grid, init=cash.payoff_grid)
    assert abs_max(f, ref_f) <= FP64_TOL
    g = cash.payoff_grid(p)
    import torch
    for n in range(10):
        g = host(s.apply(pr.PR_OP_COARSE, n, torch.from_numpy(g).cuda()))
    ref_g = im.serial_fine(p, 10, 1.0, 1, ring=cash.ring_grid, init=cash.payoff_grid)
    assert abs_max(g, ref_g) <= FP64_TOL
    ex = cash.exact_grid(p, 1.0)
    print("rel l2 vs closed form: F %.3e, G %.3e" % (cash.rel_l2(f, ex), cash.rel_l2(g, ex)))
    assert abs(cash.rel_l2(f, ex) - cash.rel_l2(ref_f, ex)) < 1e-9
    s.close()


@pytest.mark.parametrize("k", [1, 2])
def test_paper_parareal_vs_oracle(pr, k):
    """Parareal, Eq. (parareal), on the paper's problem with both propagators
    implicit on the same grid, after k iterations, against the oracle driver."""
    inst = paper_benchmark(spacing=2.0, krylov_tol=1e-13)   # 151^2 keeps the oracle quick
    p = cprob(inst)
    say("cash parareal", k)
    s = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT, coarse_kind=pr.PR_G_IMPLICIT, max_iters=k)
    res = s.solve()
    M, dT = inst.M, 0.1
    Fn = lambda n, v: im.fine(p, 3, dT / 3, n * dT, v.reshape(M, M), ring=cash.ring_grid)
    Gn = lambda n, v: im.fine(p, 1, dT, n * dT, v.reshape(M, M), ring=cash.ring_grid)
    U, K, inc = oracle.parareal_generic(cash.payoff_grid(p), 10, Fn, Gn, max_iters=k, tol=0.0)
    assert res.iters == K == k
    assert abs_max(host(res.value), U[-1].reshape(M, M)) <= FP64_TOL
    assert np.allclose(res.increments, inc, rtol=1e-6)
    s.close()


def test_paper_parareal_finite_termination_bitwise(pr):
    inst = paper_benchmark(spacing=2.0)
    say("cash finite termination")
    s = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT, coarse_kind=pr.PR_G_IMPLICIT)
    res = s.solve()
    ser = host(s.serial_fine().value)
    assert res.iters == inst.n_slices
    assert np.array_equal(host(res.value), ser)
    s.close()


def test_paper_parareal_lod_coarse(pr):
    """The same-grid direction-split coarse propagator on the paper's problem:
    finite termination bitwise, and the error against serial F at least halves
    with each of the first iterations (measured: about 3.7 times per iteration
    at 151^2)."""
    inst = paper_benchmark(spacing=2.0)
    say("cash parareal, LOD coarse")
    ser = None
    errs = []
    for k in (1, 2, 3, inst.n_slices):
        s = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT, coarse_kind=pr.PR_G_LOD, max_iters=k)
        if ser is None:
            ser = host(s.serial_fine().value)
        v = host(s.solve().value)
        errs.append(abs_max(v, ser))
        s.close()
    print("LOD-G Parareal error vs serial F at K = 1, 2, 3, N:", errs)
    assert errs[-1] == 0.0
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1]
