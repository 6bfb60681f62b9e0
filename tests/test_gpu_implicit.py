"""Implicit-Euler fine propagator (Eq. (fd), Sec. 3.2) on the GPU, by BiCGStab,
against the oracle's direct solve of the same steps.

FP64 throughout; the Krylov tolerance is 1e-13 relative residual, so the GPU
states agree with the oracle's to 1e-10 absolute.  Finite termination (K = N)
equals the GPU's serial F bitwise: every dot product is summed in a fixed order.
"""
import numpy as np
import pytest

import oracle
from oracle import implicit as im
from helpers import abs_max, oproblem, say
from synthetic import BASKET, EXCHANGE, plain_fp64

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


def implicit_inst(payoff=BASKET, **kw):
    base = dict(implicit=True, krylov_tol=1e-13, fine_steps_per_slice=4, n_slices=4,
                coarse_steps_per_slice=0, tol=0.0)
    base.update(kw)
    return plain_fp64(payoff).replace(**base)


@pytest.mark.parametrize("M,payoff,bc", [(65, BASKET, 0), (97, BASKET, 0), (129, EXCHANGE, 2)])
def test_serial_implicit_fine_vs_oracle(pr, M, payoff, bc):
    """dt = 1/16: about 60 (65^2) to 250 (129^2) times the explicit bound."""
    inst = implicit_inst(payoff, M=M, coarse_M=33)
    say("implicit serial F", M, payoff, bc)
    s = pr.Solver(inst, bc_kind=bc)
    r = s.serial_fine()
    ref = im.serial_fine(oproblem(inst, bc_kind=bc), inst.n_slices, inst.T, 4)
    err = abs_max(host(r.value), ref)
    print("max |gpu - oracle| =", err, "Krylov iterations", r.stats["krylov_iters"],
          "max per step", r.stats["krylov_max_step"])
    assert err <= FP64_TOL
    assert r.stats["krylov_unconverged"] == 0
    assert 0 < r.stats["krylov_max_step"] < 1000
    s.close()


@pytest.mark.parametrize("k", [1, 2])
def test_parareal_implicit_fine_vs_oracle(pr, k):
    """Parareal with the implicit F and the numerical G (33^2, explicit) after k
    iterations, against the oracle's Parareal driver with the same propagators."""
    inst = implicit_inst(M=65, coarse_M=33, coarse_steps_per_slice=64)
    say("implicit parareal", k)
    s = pr.Solver(inst, max_iters=k)
    res = s.solve()
    pf, pc = oproblem(inst), oproblem(inst, 33)
    dT = inst.T / inst.n_slices
    Fn = lambda n, v: im.fine(pf, 4, dT / 4, n * dT, v.reshape(65, 65))
    Gn = lambda n, v: oracle.coarse(pf, pc, 64, dT / 64, n * dT, v.reshape(65, 65))
    U, K, inc = oracle.parareal_generic(oracle.payoff_grid(pf), inst.n_slices, Fn, Gn,
                                        max_iters=k, tol=0.0)
    assert res.iters == K == k
    assert abs_max(host(res.value), U[-1].reshape(65, 65)) <= FP64_TOL
    assert np.allclose(res.increments, inc, rtol=1e-6)
    s.close()


@pytest.mark.parametrize("coarse", ["numerical", "lod"])
def test_implicit_finite_termination_bitwise(pr, coarse):
    kw = dict(M=97, coarse_M=49, coarse_steps_per_slice=0)
    kind = pr.PR_G_NUMERICAL
    if coarse == "lod":
        kw["coarse_steps_per_slice"] = 2
        kind = pr.PR_G_LOD
    inst = implicit_inst(n_slices=6, **kw)
    say("implicit finite termination", coarse)
    s = pr.Solver(inst, coarse_kind=kind)
    res = s.solve()
    ser = host(s.serial_fine().value)
    assert res.iters == inst.n_slices
    assert np.array_equal(host(res.value), ser)
    s.close()


def test_implicit_lod_coarse_converges_fast(pr):
    """The paper's pairing (Sec. 3.2): an implicit fine step three times finer
    than the implicit coarse step; with the same-grid LOD coarse propagator the
    increments fall below 1e-8 well before K = N."""
    inst = implicit_inst(M=129, coarse_M=33, n_slices=10, fine_steps_per_slice=3,
                         coarse_steps_per_slice=1, tol=1e-8)
    say("implicit fine + LOD coarse")
    s = pr.Solver(inst, coarse_kind=pr.PR_G_LOD)
    res = s.solve()
    ser = host(s.serial_fine().value)
    print("K", res.iters, "increments", res.increments)
    assert res.iters < inst.n_slices
    assert abs_max(host(res.value), ser) <= 1e-7
    s.close()
