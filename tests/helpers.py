"""Shared test helpers (no method arithmetic): instance -> oracle problem, norms."""
import sys

import numpy as np

import oracle


def oproblem(inst, M=None, bc_kind=oracle.BC_FORWARD_INTRINSIC):
    return oracle.Problem(M=M or inst.M, sigma1=inst.sigma1, sigma2=inst.sigma2, rho=inst.rho,
                          r=inst.r, payoff_kind=inst.payoff, w1=inst.w1, w2=inst.w2,
                          strike=inst.strike, bc_kind=bc_kind, s_max=inst.s_max)


def rel_max(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / np.abs(b).max())


def abs_max(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())


def say(*args):
    """Name the case on stdout before a GPU step (survives a lost box)."""
    print("[case]", *args, flush=True)
    sys.stdout.flush()
