"""Same-grid LOD coarse propagator on the GPU against the oracle."""
import numpy as np
import pytest

import oracle
from helpers import abs_max, oproblem, rel_max, say
from synthetic import BASKET, EXCHANGE, plain_at_scale, plain_fp64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pr():
    import torch
    assert torch.cuda.is_available()
    import paper_2404_02521_amd as pr_
    return pr_


def host(t):
    return t.detach().cpu().numpy()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("M,mG", [(65, 2), (67, 3), (129, 1)])
def test_lod_apply_fp64(pr, M, mG):
    inst = plain_fp64(BASKET).replace(M=M, coarse_steps_per_slice=mG, fine_steps_per_slice=0,
                                      rho=-0.4)
    mF, _, _, _ = pr.plan(inst, coarse_kind=pr.PR_G_LOD)
    p = oproblem(inst)
    dT = inst.T / inst.n_slices
    u = oracle.fine(p, mF, dT / mF, 0.0, oracle.payoff_grid(p))
    say("lod apply fp64", M, mG)
    s = pr.Solver(inst, coarse_kind=pr.PR_G_LOD)
    g = host(s.apply(pr.PR_OP_COARSE, 1, to_dev(u)))
    assert abs_max(g, oracle.lod(p, mG, dT / mG, dT, u)) <= 1e-12


@pytest.mark.parametrize("payoff", [BASKET, EXCHANGE])
@pytest.mark.parametrize("k", [1, 3])
def test_lod_parareal_fp64(pr, payoff, k):
    inst = plain_fp64(payoff).replace(tol=0.0, coarse_steps_per_slice=2)
    say("lod parareal fp64", payoff, k)
    s = pr.Solver(inst, coarse_kind=pr.PR_G_LOD, max_iters=k)
    res = s.solve()
    p = oproblem(inst)
    U, K, inc = oracle.parareal_bs(p, p, 8, 1.0, 128, 2, coarse_kind=oracle.G_LOD,
                                   max_iters=k, tol=0.0)
    assert res.iters == K == k
    assert abs_max(host(res.value), U) <= 1e-10
    assert np.allclose(res.increments, inc, rtol=1e-8, atol=1e-14)


def test_lod_parareal_fp32_vs_oracle(pr):
    inst = plain_at_scale(2, M=129, n_slices=16).replace(tol=0.0, coarse_steps_per_slice=2)
    mF, _, _, _ = pr.plan(inst, coarse_kind=pr.PR_G_LOD)
    say("lod parareal fp32 129")
    s = pr.Solver(inst, coarse_kind=pr.PR_G_LOD, max_iters=3)
    res = s.solve()
    p = oproblem(inst)
    U, K, inc = oracle.parareal_bs(p, p, 16, inst.T, mF, 2, coarse_kind=oracle.G_LOD,
                                   max_iters=3, tol=0.0)
    assert res.iters == 3
    assert rel_max(host(res.value), U) <= 1e-5
    assert np.allclose(res.increments, inc, rtol=1e-2)


@pytest.mark.parametrize("seed", [0, 4])
def test_lod_full_size_converges(pr, seed):
    """513^2 x 64 slices: few iterations to the 1e-7 relative tolerance, error vs
    serial F within 1e-5."""
    inst = plain_at_scale(seed).replace(tol=1e-7)
    say("lod full size", seed)
    s = pr.Solver(inst, coarse_kind=pr.PR_G_LOD)
    res = s.solve()
    ser = host(s.serial_fine().value)
    err = rel_max(host(res.value), ser)
    assert res.iters <= 12, res.increments
    assert err <= 1e-5, err


def test_lod_graph_replay(pr):
    import torch
    inst = plain_at_scale(1, M=129, n_slices=16)
    say("lod graph")
    e = pr.Solver(inst, coarse_kind=pr.PR_G_LOD).solve()
    s = pr.Solver(inst, coarse_kind=pr.PR_G_LOD, flags=pr.PR_FLAG_GRAPH)
    for _ in range(3):
        r = s.solve()
        torch.cuda.synchronize()
        assert r.iters == e.iters and np.array_equal(host(r.value), host(e.value))


def test_lod_max_size_2049(pr):
    """One LOD step on the largest grid the line solver takes (2047 unknowns per
    line, 2048-entry cyclic reduction) against the oracle's Thomas solves."""
    from synthetic import largest_single
    inst = largest_single().replace(n_slices=1, T=1e-3, fine_steps_per_slice=0,
                                    coarse_steps_per_slice=1, fp32=False)
    p = oproblem(inst)
    u0 = oracle.payoff_grid(p)
    say("lod max size 2049")
    s = pr.Solver(inst, coarse_kind=pr.PR_G_LOD)
    got = host(s.apply(pr.PR_OP_COARSE, 0, to_dev(u0)))
    ref = oracle.lod(p, 1, inst.T, 0.0, u0)
    assert abs_max(got, ref) <= 1e-12
    s.close()


def test_lod_solvers_of_several_sizes(pr):
    """Solvers of several grid sizes in one process: the 2049^2 line solver
    (the largest LDS footprint) and the 513^2 two-column x stage still give
    their first results bitwise after smaller LOD solvers have been created
    (each creation sets the kernels' shared-memory limit)."""
    from synthetic import largest_single
    big = largest_single().replace(n_slices=1, T=1e-3, fine_steps_per_slice=0,
                                   coarse_steps_per_slice=1, fp32=False)
    mid = plain_at_scale(3, M=513, n_slices=2, coarse_M=129).replace(T=0.01, fp32=False)
    say("lod solvers of several sizes")
    sb = pr.Solver(big, coarse_kind=pr.PR_G_LOD)
    sm = pr.Solver(mid, coarse_kind=pr.PR_G_LOD)
    ub, um = to_dev(oracle.payoff_grid(oproblem(big))), to_dev(oracle.payoff_grid(oproblem(mid)))
    gb0 = host(sb.apply(pr.PR_OP_COARSE, 0, ub))
    gm0 = host(sm.apply(pr.PR_OP_COARSE, 0, um))
    small = [pr.Solver(plain_fp64(BASKET).replace(M=M, fine_steps_per_slice=0,
                                                  coarse_steps_per_slice=0),
                       coarse_kind=pr.PR_G_LOD)
             for M in (33, 65, 129)]
    assert np.array_equal(host(sb.apply(pr.PR_OP_COARSE, 0, ub)), gb0)
    assert np.array_equal(host(sm.apply(pr.PR_OP_COARSE, 0, um)), gm0)
    for s in small + [sb, sm]:
        s.close()
