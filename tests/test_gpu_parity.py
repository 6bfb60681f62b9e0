"""GPU path (through the C ABI) against the FP64 oracle, element by element.

Tolerances: FP64 runs within 1e-10 absolute of the oracle; FP32 runs (FP32
increments over an FP64 base, FP64 correction and norm) within 1e-5 relative
max-norm of the FP64 oracle.  Bitwise properties (finite termination, G = F,
determinism) compare the GPU with itself.
"""
import numpy as np
import pytest

import oracle
from helpers import abs_max, oproblem, rel_max, say
from synthetic import BASKET, EXCHANGE, plain_at_scale, plain_fp64

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-5


@pytest.fixture(scope="module")
def pr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2404_02521_amd as pr_
    return pr_


def host(t):
    return t.detach().cpu().numpy()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


# ---------------------------------------------------------------- fine propagator
@pytest.mark.parametrize("payoff", [BASKET, EXCHANGE])
def test_c1_serial_fine_fp64(pr, payoff):
    inst = plain_fp64(payoff)
    say("c1 serial F fp64", payoff)
    s = pr.Solver(inst)
    gpu = host(s.serial_fine().value)
    ref = oracle.serial_fine(oproblem(inst), inst.n_slices, inst.T, inst.fine_steps_per_slice)
    assert abs_max(gpu, ref) <= FP64_TOL


def test_apply_fine_and_coarse_fp64(pr):
    inst = plain_fp64(BASKET)
    pf, pc = oproblem(inst), oproblem(inst, inst.coarse_M)
    dT = inst.T / inst.n_slices
    u = oracle.payoff_grid(pf)
    for n in range(3):
        u = oracle.fine(pf, 128, dT / 128, n * dT, u)
    say("apply F/G fp64 slice 3")
    s = pr.Solver(inst)
    f_gpu = host(s.apply(pr.PR_OP_FINE, 3, to_dev(u)))
    g_gpu = host(s.apply(pr.PR_OP_COARSE, 3, to_dev(u)))
    f_ref = oracle.fine(pf, 128, dT / 128, 3 * dT, u)
    g_ref = oracle.coarse(pf, pc, 64, dT / 64, 3 * dT, u)
    assert abs_max(f_gpu, f_ref) <= 1e-12
    assert abs_max(g_gpu, g_ref) <= 1e-12


@pytest.mark.parametrize("M,Mc,N", [(5, 3, 2), (67, 23, 3), (97, 33, 2), (131, 27, 2)])
def test_ragged_grids_fp64(pr, M, Mc, N):
    """Grids that are not 2^k + 1: partial wavefront strips and row chunks; step
    counts from the planner (0.9 of the Gershgorin bound)."""
    inst = plain_fp64(BASKET).replace(M=M, coarse_M=Mc, fine_steps_per_slice=0,
                                      coarse_steps_per_slice=0, n_slices=N, sigma2=0.25,
                                      rho=-0.4, T=0.5)
    mF, mG, _, _ = pr.plan(inst)
    say("ragged fp64", M, Mc, mF, mG)
    s = pr.Solver(inst)
    ser = host(s.serial_fine().value)
    assert abs_max(ser, oracle.serial_fine(oproblem(inst), N, inst.T, mF)) <= FP64_TOL
    res = s.solve()
    U, K, _ = oracle.parareal_bs(oproblem(inst), oproblem(inst, Mc), N, inst.T, mF, mG,
                                 tol=inst.tol)
    assert res.iters == K
    assert abs_max(host(res.value), U) <= FP64_TOL


@pytest.mark.parametrize("fp32", [False, True])
@pytest.mark.parametrize("fuse", [1, 2, 3, 4, 5, 6, 7, 8])
def test_every_fused_step_count(pr, monkeypatch, fuse, fp32):
    """Every fused-step count S = 1..8 of the temporally blocked step kernel (and
    the remainder launch: 3 x 23 steps leave 23 mod S) on a ragged grid whose
    strips of 64 - 2S columns and row chunks end part-way, F over three slices
    against the oracle's serial F."""
    monkeypatch.setenv("PR_STEP_FUSE", str(fuse))
    monkeypatch.setenv("PR_STEP_SMALL_COUNT", "0")
    monkeypatch.setenv("PR_STEP_MINROWS", "5")
    inst = plain_fp64(EXCHANGE).replace(M=151, coarse_M=31, n_slices=3, fine_steps_per_slice=23,
                                        coarse_steps_per_slice=2, T=0.012, fp32=fp32)
    say("fused step count", fuse, fp32)
    s = pr.Solver(inst)
    gpu = host(s.serial_fine().value)
    ref = oracle.serial_fine(oproblem(inst), 3, inst.T, 23)
    if fp32:
        assert rel_max(gpu, ref) <= FP32_TOL
    else:
        assert abs_max(gpu, ref) <= FP64_TOL
    s.close()


@pytest.mark.parametrize("fp32", [False, True])
def test_launch_geometry_is_bitwise_invisible(pr, monkeypatch, fp32):
    """Every point-step is the same expression whatever the launch geometry, so
    serial F is bitwise the same for every fused-step count S and row-chunk size
    (interior, one-ring-column and general row paths, remainder launches)."""
    inst = plain_fp64(BASKET).replace(M=131, coarse_M=27, n_slices=2, fine_steps_per_slice=0,
                                      coarse_steps_per_slice=0, T=0.03, fp32=fp32)
    outs = []
    for fuse, rows in [(1, 0), (3, 0), (6, 0), (8, 0), (6, 5), (4, 64)]:
        monkeypatch.setenv("PR_STEP_FUSE", str(fuse))
        monkeypatch.setenv("PR_STEP_SMALL_COUNT", "0")
        monkeypatch.setenv("PR_STEP_ROWS", str(rows))
        say("launch geometry", fp32, fuse, rows)
        s = pr.Solver(inst)
        outs.append(host(s.serial_fine().value))
        s.close()
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_exact_bc_fp64(pr):
    """Margrabe ring (exchange) through the closed-form ring path."""
    inst = plain_fp64(EXCHANGE)
    say("exact bc fp64")
    s = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT)
    gpu = host(s.serial_fine().value)
    ref = oracle.serial_fine(oproblem(inst, bc_kind=oracle.BC_EXACT), 8, 1.0, 128)
    assert abs_max(gpu, ref) <= FP64_TOL


@pytest.mark.parametrize("fp32", [False, True])
def test_discounted_payoff_bc(pr, fp32):
    """The literal discounted-payoff ring (e^{-r tau} times the payoff) through
    serial F and two Parareal iterations, against the oracle."""
    inst = plain_fp64(BASKET).replace(M=129, coarse_M=33, fine_steps_per_slice=0,
                                      coarse_steps_per_slice=0, T=0.25, n_slices=4, tol=0.0,
                                      fp32=fp32)
    mf, mg, _, _ = pr.plan(inst)
    say("discounted payoff bc", fp32, mf, mg)
    s = pr.Solver(inst, bc_kind=pr.PR_BC_DISCOUNTED_PAYOFF, max_iters=2)
    pf = oproblem(inst, bc_kind=oracle.BC_DISCOUNTED_PAYOFF)
    pc = oproblem(inst, inst.coarse_M, bc_kind=oracle.BC_DISCOUNTED_PAYOFF)
    ser = host(s.serial_fine().value)
    ref = oracle.serial_fine(pf, 4, inst.T, mf)
    res = s.solve()
    U, K, _ = oracle.parareal_bs(pf, pc, 4, inst.T, mf, mg, max_iters=2, tol=0.0)
    assert res.iters == K == 2
    if fp32:
        assert rel_max(ser, ref) <= FP32_TOL
        assert rel_max(host(res.value), U) <= FP32_TOL
    else:
        assert abs_max(ser, ref) <= FP64_TOL
        assert abs_max(host(res.value), U) <= FP64_TOL
    s.close()


@pytest.mark.parametrize("M", [131, 257])
def test_exact_bc_fp32(pr, M):
    """Margrabe ring (exchange) in the FP32 increment form: the closed-form ring
    values of the edge strips' row path (evaluated three rows at a time across
    lanes) and of the ring rows, against the oracle's serial F."""
    inst = plain_fp64(EXCHANGE).replace(M=M, fp32=True, fine_steps_per_slice=0,
                                        coarse_steps_per_slice=0, T=0.05, n_slices=2,
                                        coarse_M=(M - 1) // 2 + 1)
    mf, _, _, _ = pr.plan(inst)
    say("exact bc fp32", M, mf)
    s = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT)
    gpu = host(s.serial_fine().value)
    ref = oracle.serial_fine(oproblem(inst, bc_kind=oracle.BC_EXACT), 2, inst.T, mf)
    assert rel_max(gpu, ref) <= FP32_TOL
    s.close()


@pytest.mark.parametrize("M", [5, 33, 67])
def test_narrow_grids_fp32(pr, M):
    """Grids narrower than a wavefront strip (both ring columns in one strip, the
    general row path throughout) and one just wider, FP32 increment form, serial F
    against the oracle."""
    inst = plain_fp64(BASKET).replace(M=M, fp32=True, fine_steps_per_slice=0,
                                      coarse_steps_per_slice=0, T=0.2, n_slices=2,
                                      coarse_M=(M - 1) // 2 + 1)
    mf, _, _, _ = pr.plan(inst)
    say("narrow fp32", M, mf)
    s = pr.Solver(inst)
    gpu = host(s.serial_fine().value)
    ref = oracle.serial_fine(oproblem(inst), 2, inst.T, mf)
    assert rel_max(gpu, ref) <= FP32_TOL
    s.close()


# ---------------------------------------------------------------- Parareal, FP64
@pytest.mark.parametrize("payoff", [BASKET, EXCHANGE])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_c1_parareal_iterates_fp64(pr, payoff, k):
    inst = plain_fp64(payoff).replace(tol=0.0)
    say("c1 parareal fp64", payoff, k)
    s = pr.Solver(inst, max_iters=k)
    res = s.solve()
    U, K, inc = oracle.parareal_bs(oproblem(inst), oproblem(inst, inst.coarse_M), 8, 1.0, 128,
                                   64, max_iters=k, tol=0.0)
    assert res.iters == K == k
    assert abs_max(host(res.value), U) <= FP64_TOL
    assert np.allclose(res.increments, inc, rtol=1e-8, atol=1e-13)


@pytest.mark.parametrize("payoff", [BASKET, EXCHANGE])
def test_c1_parareal_full_fp64(pr, payoff):
    inst = plain_fp64(payoff)
    say("c1 parareal full fp64", payoff)
    s = pr.Solver(inst)
    res = s.solve()
    ser = host(s.serial_fine().value)
    U, K, _ = oracle.parareal_bs(oproblem(inst), oproblem(inst, inst.coarse_M), 8, 1.0, 128, 64,
                                 tol=inst.tol)
    assert res.iters == K
    assert abs_max(host(res.value), U) <= FP64_TOL
    if K == inst.n_slices:
        assert np.array_equal(host(res.value), ser)


@pytest.mark.parametrize("fp32", [False, True])
def test_finite_termination_bitwise(pr, fp32):
    inst = plain_fp64(BASKET).replace(tol=0.0, fp32=fp32)
    say("finite termination", fp32)
    s = pr.Solver(inst)
    res = s.solve()
    assert res.iters == inst.n_slices
    assert np.array_equal(host(res.value), host(s.serial_fine().value))


@pytest.mark.parametrize("fp32", [False, True])
def test_finite_termination_bitwise_mixed_fused_steps(pr, monkeypatch, fp32):
    """With sweeps of <= 4 slices (and serial F) on S = 3 and larger sweeps on
    S = 6, Parareal after N iterations still equals serial F bitwise."""
    monkeypatch.setenv("PR_STEP_FUSE", "6")
    monkeypatch.setenv("PR_STEP_FUSE_SMALL", "3")
    monkeypatch.setenv("PR_STEP_SMALL_COUNT", "4")
    inst = plain_fp64(BASKET).replace(tol=0.0, fp32=fp32)
    say("finite termination mixed S", fp32)
    s = pr.Solver(inst)
    res = s.solve()
    assert res.iters == inst.n_slices
    assert np.array_equal(host(res.value), host(s.serial_fine().value))
    s.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_finite_termination_bitwise_bench_shape(pr, seed):
    """The at-scale workload itself (513^2 FP32 increments, N = 64, numerical G on
    the compiled-in 129^2 chain, sweeps over 64 slices on other row chunks than
    serial F's): with tol = 0 the iteration runs to K = N and equals serial F
    bitwise (seed 0 differed in the last bits while multiply-adds could fuse
    across statements)."""
    inst = plain_at_scale(seed).replace(tol=0.0)
    say("finite termination bench shape", seed)
    s = pr.Solver(inst)
    ser = host(s.serial_fine().value)
    res = s.solve()
    assert res.iters == inst.n_slices
    assert np.array_equal(host(res.value), ser)
    s.close()


def test_bench_shape_chain_vs_oracle(pr):
    """513^2 / 129^2 FP32 (the compiled-in LDS chain) over Parareal iterations
    k = 1, 2 against the oracle's Parareal, 4 slices of the at-scale length."""
    inst = plain_at_scale(0).replace(n_slices=4, T=4.0 / 64, tol=0.0)
    mf, mg, _, _ = pr.plan(inst)
    say("bench shape chain vs oracle", mf, mg)
    for k in (1, 2):
        s = pr.Solver(inst, max_iters=k)
        res = s.solve()
        U, K, inc = oracle.parareal_bs(oproblem(inst), oproblem(inst, 129), 4, inst.T, mf, mg,
                                       max_iters=k, tol=0.0)
        assert res.iters == K == k
        assert rel_max(host(res.value), U) <= FP32_TOL
        assert np.allclose(res.increments, inc, rtol=1e-3)
        s.close()


@pytest.mark.parametrize("fp32", [False, True])
def test_G_equal_F_one_iteration(pr, fp32):
    inst = plain_fp64(EXCHANGE).replace(fp32=fp32)
    say("G=F", fp32)
    s = pr.Solver(inst, coarse_kind=pr.PR_G_FINE)
    res = s.solve()
    assert res.iters == 1 and res.increments[0] == 0.0
    assert np.array_equal(host(res.value), host(s.serial_fine().value))


def test_single_slice(pr):
    inst = plain_fp64(BASKET).replace(n_slices=1, fine_steps_per_slice=1024,
                                      coarse_steps_per_slice=512)
    say("N=1")
    s = pr.Solver(inst)
    res = s.solve()
    assert res.iters == 1
    assert np.array_equal(host(res.value), host(s.serial_fine().value))


def test_deterministic(pr):
    inst = plain_at_scale(3, M=129, n_slices=16, coarse_M=33)
    say("determinism")
    s = pr.Solver(inst, max_iters=3)
    a = host(s.solve().value)
    b = host(s.solve().value)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- FP32 increments
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fp32_serial_fine_vs_oracle(pr, seed):
    inst = plain_at_scale(seed, M=129, n_slices=8, coarse_M=33)
    mf, mg, _, _ = pr.plan(inst)
    say("fp32 serial F 129", seed, mf)
    s = pr.Solver(inst)
    gpu = host(s.serial_fine().value)
    ref = oracle.serial_fine(oproblem(inst), 8, inst.T, mf)
    assert rel_max(gpu, ref) <= FP32_TOL


@pytest.mark.parametrize("seed", [0, 4])
def test_fp32_parareal_vs_oracle(pr, seed):
    inst = plain_at_scale(seed, M=129, n_slices=8, coarse_M=33).replace(tol=0.0)
    mf, mg, _, _ = pr.plan(inst)
    say("fp32 parareal 129", seed)
    for k in (1, 3):
        s = pr.Solver(inst, max_iters=k)
        res = s.solve()
        U, K, inc = oracle.parareal_bs(oproblem(inst), oproblem(inst, 33), 8, inst.T, mf, mg,
                                       max_iters=k, tol=0.0)
        assert res.iters == K == k
        assert rel_max(host(res.value), U) <= FP32_TOL
        assert np.allclose(res.increments, inc, rtol=1e-3)


@pytest.mark.parametrize("fp32,M,Mc", [(True, 513, 257), (False, 257, 129)])
def test_coarse_chain_state_in_global_memory(pr, fp32, M, Mc):
    """Coarse grids whose stepped state does not fit in LDS (FP32 257^2, FP64
    129^2) run the chain with its two state buffers in global memory: Parareal
    iterates k = 1, 2 against the oracle."""
    inst = plain_at_scale(3, M=M, n_slices=4, coarse_M=Mc).replace(T=0.04, tol=0.0, fp32=fp32)
    mf, mg, _, _ = pr.plan(inst)
    say("chain state in global memory", fp32, M, Mc, mf, mg)
    for k in (1, 2):
        s = pr.Solver(inst, max_iters=k)
        res = s.solve()
        U, K, inc = oracle.parareal_bs(oproblem(inst), oproblem(inst, Mc), 4, inst.T, mf, mg,
                                       max_iters=k, tol=0.0)
        assert res.iters == K == k
        if fp32:
            assert rel_max(host(res.value), U) <= FP32_TOL
            assert np.allclose(res.increments, inc, rtol=1e-3)
        else:
            assert abs_max(host(res.value), U) <= FP64_TOL
            assert np.allclose(res.increments, inc, rtol=1e-8, atol=1e-14)
        s.close()


def test_full_size_fine_slice_vs_oracle(pr):
    """513^2 at the at-scale launch shape: F over slice 0 (planned steps) and G over
    slice 0 (129^2 coarse grid), checked against the oracle."""
    inst = plain_at_scale(0)
    mf, mg, _, _ = pr.plan(inst)
    pf, pc = oproblem(inst), oproblem(inst, inst.coarse_M)
    dT = inst.T / inst.n_slices
    u0 = oracle.payoff_grid(pf)
    say("full-size F/G slice 0", mf, mg)
    s = pr.Solver(inst)
    f_gpu = host(s.apply(pr.PR_OP_FINE, 0, to_dev(u0)))
    g_gpu = host(s.apply(pr.PR_OP_COARSE, 0, to_dev(u0)))
    assert rel_max(f_gpu, oracle.fine(pf, mf, dT / mf, 0.0, u0)) <= FP32_TOL
    assert rel_max(g_gpu, oracle.coarse(pf, pc, mg, dT / mg, 0.0, u0)) <= FP32_TOL


def test_full_size_parareal_error_vs_serial(pr):
    """At-scale solve: the returned error against serial F is what the stop rule allows."""
    inst = plain_at_scale(3)
    say("full-size parareal seed 3")
    s = pr.Solver(inst)
    res = s.solve()
    ser = host(s.serial_fine().value)
    err = rel_max(host(res.value), ser)
    assert res.iters >= 1
    assert err <= FP32_TOL, (res.iters, err)


def test_max_size_fused_launch_2049(pr, monkeypatch):
    """The largest grid (2049^2) through exactly one prep step plus one 6-step
    fused launch of the FP32 increment kernel, against the FP64 oracle; the
    increment F(u) - u is checked on its own scale."""
    from synthetic import largest_single
    monkeypatch.setenv("PR_STEP_FUSE", "6")
    monkeypatch.setenv("PR_STEP_SMALL_COUNT", "0")
    inst = largest_single().replace(n_slices=1, T=7e-6, fine_steps_per_slice=7,
                                    coarse_steps_per_slice=1)
    p = oproblem(inst)
    u0 = oracle.payoff_grid(p)
    say("max size 2049 fused launch")
    s = pr.Solver(inst, coarse_kind=pr.PR_G_LOD)
    got = host(s.apply(pr.PR_OP_FINE, 0, to_dev(u0)))
    ref = oracle.fine(p, 7, inst.T / 7, 0.0, u0)
    assert rel_max(got, ref) <= FP32_TOL
    assert rel_max(got - u0, ref - u0) <= FP32_TOL
    s.close()
