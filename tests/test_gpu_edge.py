"""Degenerate cases of the method on the GPU against the oracle: parameters at
the edges of the model (no correlation, correlation near +-1, no interest rate,
a volatility small enough that the drift dominates the diffusion near the far
edge, a maturity of one step), the smallest implicit problem (3 x 3
unknowns), and the smallest three-asset problem with a single slice."""
import numpy as np
import pytest

import oracle
from helpers import abs_max, oproblem, say
from oracle import implicit as im
from oracle import nasset as na
from synthetic import BASKET, EXCHANGE, plain_fp64, three_asset

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


CASES = {
    "rho0": dict(rho=0.0),
    "rho+0.95": dict(rho=0.95),
    "rho-0.95": dict(rho=-0.95),
    "r0": dict(r=0.0),
    "sigma_small": dict(sigma1=0.02, sigma2=0.03, r=0.1),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("payoff", [BASKET, EXCHANGE])
def test_degenerate_parameters(pr, case, payoff):
    """49^2 over 25^2, N = 4, planned step counts: serial F and two Parareal
    iterations against the oracle."""
    inst = plain_fp64(payoff).replace(M=49, coarse_M=25, n_slices=4, T=0.5,
                                      fine_steps_per_slice=0, coarse_steps_per_slice=0,
                                      tol=0.0, **CASES[case])
    mF, mG, _, _ = pr.plan(inst)
    say("degenerate", case, payoff, mF, mG)
    s = pr.Solver(inst, max_iters=2)
    ser = host(s.serial_fine().value)
    assert abs_max(ser, oracle.serial_fine(oproblem(inst), 4, inst.T, mF)) <= FP64_TOL
    res = s.solve()
    U, K, _ = oracle.parareal_bs(oproblem(inst), oproblem(inst, 25), 4, inst.T, mF, mG,
                                 max_iters=2, tol=0.0)
    assert res.iters == K == 2
    assert abs_max(host(res.value), U) <= FP64_TOL
    s.close()


def test_one_step_maturity(pr):
    """T equal to a single explicit step per slice on each grid."""
    base = plain_fp64(BASKET).replace(M=33, coarse_M=17, n_slices=2)
    inst = base.replace(T=2e-4, fine_steps_per_slice=1, coarse_steps_per_slice=1)
    say("one-step maturity")
    s = pr.Solver(inst)
    ser = host(s.serial_fine().value)
    assert abs_max(ser, oracle.serial_fine(oproblem(inst), 2, inst.T, 1)) <= FP64_TOL
    res = s.solve()
    assert res.iters <= 2
    s.close()


def test_smallest_implicit_problem(pr):
    """5^2 nodes (3 x 3 unknowns), implicit F with dt far above the explicit
    bound, N = 2: serial F against the oracle's direct solve, and finite
    termination."""
    inst = plain_fp64(BASKET).replace(M=5, coarse_M=3, n_slices=2, T=1.0, implicit=True,
                                      krylov_tol=1e-14, fine_steps_per_slice=2,
                                      coarse_steps_per_slice=0, tol=0.0)
    say("smallest implicit")
    s = pr.Solver(inst)
    r = s.serial_fine()
    ref = im.serial_fine(oproblem(inst), 2, 1.0, 2)
    assert abs_max(host(r.value), ref) <= FP64_TOL
    assert r.stats["krylov_unconverged"] == 0
    res = s.solve()
    assert res.iters == 2 and np.array_equal(host(res.value), host(r.value))
    s.close()


def test_smallest_three_asset_problem(pr):
    """5^3 nodes (27 unknowns), coarse 3^3 (one unknown), one slice: serial F
    against the oracle, and Parareal's single iteration equal to it bitwise."""
    from paper_2404_02521_amd import nasset
    inst = three_asset(7, M=5, coarse_M=3, n_slices=1, T=0.05)
    say("smallest three-asset")
    s = nasset.Solver3(inst)
    v, st = s.serial_fine()
    p = na.Problem3(M=5, sigma=inst.sigma, rho=inst.rho, r=inst.r, w=inst.w,
                    strike=inst.strike, s_max=inst.s_max)
    assert abs_max(host(v), na.serial_fine(p, 1, inst.T, st["fine_steps"])) <= FP64_TOL
    u, st2 = s.solve()
    assert st2["iters"] == 1 and np.array_equal(host(u), host(v))
    s.close()
