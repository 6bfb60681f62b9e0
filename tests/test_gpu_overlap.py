"""The overlapped coarse chain (default for explicit F with the numerical G):
the fine sweep runs slice group by slice group while a second stream runs each
finished group's chain and correction, Eq. (parareal) (Sec. 3.1) unchanged.
Two schedules: equal groups (PR_PIPE_MODE 0), and phases with a fixed group
boundary whose next first-group sweep starts beside the current second-group
chain (PR_PIPE_MODE 1, the default).

Checks: bitwise equality with the serial schedule (PR_FLAG_SERIAL_CHAIN) at the
at-scale shape (513^2 FP32, N = 64, chain on 129^2) after a few iterations and
to convergence; with smaller groups forced (PR_PIPE_MIN, PR_PIPE_GROUPS) in
both schedules, the same equality, parity with the oracle's Parareal in FP64
and finite termination; a tolerance stop inside a phase (the early sweep is
discarded) followed by a second solve on the same solver.
"""
import numpy as np
import pytest

import oracle
from helpers import abs_max, oproblem, say
from synthetic import BASKET, plain_at_scale, plain_fp64

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


def both(pr, inst, **kw):
    """(overlapped result, serial-chain result) of the same solve."""
    out = []
    for flags in (0, pr.PR_FLAG_SERIAL_CHAIN):
        s = pr.Solver(inst, flags=flags, **kw)
        r = s.solve()
        out.append((host(r.value), list(r.increments), r.iters, r.stats))
        s.close()
    return out


@pytest.mark.parametrize("seed,k", [(0, 3), (3, 0)])
def test_overlap_bitwise_at_scale(pr, seed, k):
    """k = 0: to convergence (the relative stop of the at-scale problem)."""
    inst = plain_at_scale(seed)
    say("overlap bitwise at scale", seed, k)
    (a, ia, ka, sa), (b, ib, kb, sb) = both(pr, inst, max_iters=k)
    assert ka == kb
    assert ia == ib
    assert np.array_equal(a, b)
    print("iters", ka, "fine ms", sa["t_fine_ms"], "exposed chain ms", sa["t_chain_ms"],
          "| serial: fine ms", sb["t_fine_ms"], "chain ms", sb["t_chain_ms"])


@pytest.mark.parametrize("mode", ["0", "1"])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_overlap_small_groups_vs_oracle(pr, monkeypatch, k, mode):
    """65^2 FP64, N = 8: equal groups of 2 (mode 0: 4 groups, each later
    group's chain restarting from the corrected state) or phases of two groups
    down to 2 slices (mode 1): against the oracle's Parareal and bitwise
    against the serial schedule."""
    monkeypatch.setenv("PR_PIPE_MIN", "2")
    monkeypatch.setenv("PR_PIPE_GROUPS", "4")
    monkeypatch.setenv("PR_PIPE_MODE", mode)
    inst = plain_fp64(BASKET).replace(tol=0.0)
    say("overlap small groups", k)
    (a, ia, ka, _), (b, ib, _, _) = both(pr, inst, max_iters=k)
    U, K, inc = oracle.parareal_bs(oproblem(inst), oproblem(inst, inst.coarse_M), 8, 1.0, 128, 64,
                                   max_iters=k, tol=0.0)
    assert ka == K == k
    assert abs_max(a, U) <= FP64_TOL
    assert np.allclose(ia, inc, rtol=1e-8, atol=1e-13)
    assert np.array_equal(a, b) and ia == ib


@pytest.mark.parametrize("mode", ["0", "1"])
def test_overlap_small_groups_finite_termination(pr, monkeypatch, mode):
    """129^2 FP32 over 33^2, N = 16: three equal groups (mode 0: 6, 6, 4 slices
    while 16 are active; ragged groups as the active count shrinks) or phases
    with boundaries at slices 8, 12 and 14 (mode 1): K = N equals serial F
    bitwise."""
    monkeypatch.setenv("PR_PIPE_MIN", "3")
    monkeypatch.setenv("PR_PIPE_GROUPS", "3")
    monkeypatch.setenv("PR_PIPE_MODE", mode)
    inst = plain_at_scale(5, M=129, n_slices=16, coarse_M=33).replace(tol=0.0)
    say("overlap finite termination")
    s = pr.Solver(inst)
    r = s.solve()
    ser = host(s.serial_fine().value)
    assert r.iters == 16
    assert np.array_equal(host(r.value), ser)
    s.close()


def test_phased_stop_inside_a_phase(pr, monkeypatch):
    """Phases down to 2 slices, 129^2 FP32 over 33^2, N = 16 (first phase: the
    boundary at slice 8), with an absolute tolerance between the 4th and 5th
    increments of the run to K = N: the solve stops inside the first phase,
    with the next iteration's first-group sweep already issued and discarded.
    Equal to the serial schedule bitwise, and a second solve on the same solver
    repeats the first."""
    monkeypatch.setenv("PR_PIPE_MIN", "2")
    monkeypatch.setenv("PR_PIPE_MODE", "1")
    base = plain_at_scale(6, M=129, n_slices=16, coarse_M=33).replace(tol=0.0,
                                                                     tol_relative=False)
    s = pr.Solver(base, flags=pr.PR_FLAG_SERIAL_CHAIN)
    inc = list(s.solve().increments)
    s.close()
    inst = base.replace(tol=0.5 * (inc[3] + inc[4]))
    say("phased stop inside a phase", inc[:6])
    (a, ia, ka, _), (b, ib, kb, _) = both(pr, inst)
    print("iters", ka)
    assert ka == kb and 2 <= ka < 8
    assert ia == ib and np.array_equal(a, b)
    s = pr.Solver(inst)
    r1, r2 = s.solve(), s.solve()
    assert r1.iters == r2.iters == ka
    assert np.array_equal(host(r1.value), a) and np.array_equal(host(r2.value), a)
    s.close()
