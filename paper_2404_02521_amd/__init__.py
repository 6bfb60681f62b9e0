"""MI355X-native Parareal for the two-asset Black-Scholes equation.

The compute path is the gfx950 HIP library ``libparareal.so`` behind the C ABI
of ``include/parareal.h``; this package only marshals arguments and lets torch
provide device memory and streams.
"""
from . import _lib
from ._lib import (PR_BC_DISCOUNTED_PAYOFF, PR_BC_EXACT, PR_BC_FORWARD_INTRINSIC, PR_FINE_EXPLICIT,
                   PR_FINE_IMPLICIT, PR_FLAG_GRAPH, PR_FLAG_NO_FALLBACK, PR_FLAG_SERIAL_CHAIN,
                   PR_FLAG_TIME_STEPS, PR_FP32,
                   PR_FP64, PR_G_FINE, PR_G_FNO, PR_G_IMPLICIT, PR_G_LOD, PR_G_NUMERICAL,
                   PR_OP_COARSE, PR_OP_FINE, PR_PAYOFF_BASKET_CALL, PR_PAYOFF_CASH_OR_NOTHING,
                   PR_PAYOFF_EXCHANGE, PR_SERVER_RAGGED_F, PararealError)
from .parareal import Solver, SolveResult, plan

__all__ = ["Solver", "SolveResult", "plan", "PararealError", "PR_FP32", "PR_FP64",
           "PR_G_NUMERICAL", "PR_G_FNO", "PR_G_FINE", "PR_G_LOD", "PR_G_IMPLICIT", "PR_OP_FINE",
           "PR_OP_COARSE", "PR_BC_EXACT", "PR_BC_FORWARD_INTRINSIC", "PR_BC_DISCOUNTED_PAYOFF",
           "PR_PAYOFF_BASKET_CALL", "PR_PAYOFF_EXCHANGE", "PR_PAYOFF_CASH_OR_NOTHING",
           "PR_FINE_EXPLICIT", "PR_FINE_IMPLICIT", "PR_FLAG_TIME_STEPS", "PR_FLAG_GRAPH",
           "PR_FLAG_NO_FALLBACK", "PR_FLAG_SERIAL_CHAIN", "PR_SERVER_RAGGED_F", "_lib"]
