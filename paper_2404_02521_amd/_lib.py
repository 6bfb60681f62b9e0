"""ctypes binding of ``libparareal.so`` (the C ABI in include/parareal.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libparareal.so")

PR_MAX_SLICES = 1024
PR_STATIC_SCRATCH_BYTES = 64 << 20

(PR_OK, PR_EINVAL, PR_EUNSTABLE, PR_ENOMEM, PR_EDEVICE, PR_ENOTCONV, PR_ENONFINITE, PR_EMODEL,
 PR_EBUSY) = range(9)
PR_PAYOFF_BASKET_CALL, PR_PAYOFF_EXCHANGE, PR_PAYOFF_CASH_OR_NOTHING = 0, 1, 2
PR_BC_FORWARD_INTRINSIC, PR_BC_DISCOUNTED_PAYOFF, PR_BC_EXACT = 0, 1, 2
PR_G_NUMERICAL, PR_G_FNO, PR_G_FINE, PR_G_LOD, PR_G_IMPLICIT = 0, 1, 2, 3, 4
PR_FP64, PR_FP32 = 0, 1
PR_FINE_EXPLICIT, PR_FINE_IMPLICIT = 0, 1
PR_OP_FINE, PR_OP_COARSE = 0, 1
PR_FLAG_TIME_STEPS = 1
PR_FLAG_GRAPH = 2
PR_FLAG_NO_FALLBACK = 4
PR_FLAG_SERIAL_CHAIN = 8
PR_SERVER_RAGGED_F = 1
PR_FNO_FP32, PR_FNO_BF16 = 0, 1
PR_FNO_BASE_ZERO, PR_FNO_BASE_IDENTITY, PR_FNO_BASE_LOD, PR_FNO_BASE_FINE_LOD = 0, 1, 2, 3
PR_FNO_GRID = 64
PR_FNO_MAX_BATCH = 512


class pr_grid(C.Structure):
    _fields_ = [("n", C.c_int32), ("pad_", C.c_int32), ("s_max", C.c_double)]


class pr_model(C.Structure):
    _fields_ = [("sigma1", C.c_double), ("sigma2", C.c_double), ("rho", C.c_double),
                ("r", C.c_double), ("T", C.c_double)]


class pr_payoff(C.Structure):
    _fields_ = [("kind", C.c_int32), ("bc_kind", C.c_int32), ("w1", C.c_double),
                ("w2", C.c_double), ("strike", C.c_double), ("strike2", C.c_double),
                ("cash", C.c_double)]


class pr_options(C.Structure):
    _fields_ = [("n_slices", C.c_int32), ("max_iters", C.c_int32), ("tol", C.c_double),
                ("tol_relative", C.c_int32), ("precision", C.c_int32), ("fine_steps", C.c_int32),
                ("coarse_kind", C.c_int32), ("coarse_n", C.c_int32), ("coarse_steps", C.c_int32),
                ("cfl", C.c_double), ("flags", C.c_uint32), ("fine_scheme", C.c_int32),
                ("krylov_tol", C.c_double), ("krylov_max_iters", C.c_int32), ("pad2_", C.c_int32)]


class pr_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("fine_steps", C.c_int32),
                ("coarse_steps", C.c_int32), ("last_increment", C.c_double),
                ("scale", C.c_double), ("increments", C.c_double * (PR_MAX_SLICES + 1)),
                ("t_total_ms", C.c_double), ("t_fine_ms", C.c_double),
                ("t_chain_ms", C.c_double), ("t_correct_ms", C.c_double),
                ("fine_point_steps", C.c_int64), ("fine_step_launches", C.c_int64),
                ("fine_step_bytes", C.c_double), ("t_step_kernels_ms", C.c_double),
                ("workspace_bytes", C.c_uint64), ("coarse_fallback", C.c_int32),
                ("pad_", C.c_int32), ("timed_step_launches", C.c_int64),
                ("timed_step_bytes", C.c_double), ("krylov_iters", C.c_int64),
                ("krylov_max_step", C.c_int32), ("krylov_unconverged", C.c_int32)]


class pr_server_options(C.Structure):
    _fields_ = [("max_resident", C.c_int32), ("n_streams", C.c_int32), ("flags", C.c_uint32),
                ("max_queued", C.c_int32)]


class pr_fno_config(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("precision", C.c_int32), ("out_scale", C.c_double),
                ("base", C.c_int32), ("pad_", C.c_int32)]


class pr_fno_file_info(C.Structure):
    _fields_ = [("version", C.c_uint32), ("base", C.c_int32), ("precision", C.c_int32),
                ("pad_", C.c_int32), ("out_scale", C.c_double), ("param_count", C.c_uint64),
                ("train_hash", C.c_uint64)]


class pr_request_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("last_increment", C.c_double),
                ("latency_ms", C.c_double), ("queue_ms", C.c_double),
                ("workspace_bytes", C.c_uint64), ("coarse_fallback", C.c_int32),
                ("reserved_", C.c_int32)]


# (name, restype, argtypes) of every exported entry point of include/parareal.h
class pr3_problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("coarse_n", C.c_int32), ("n_slices", C.c_int32),
                ("max_iters", C.c_int32), ("fine_steps", C.c_int32), ("coarse_steps", C.c_int32),
                ("s_max", C.c_double), ("T", C.c_double), ("tol", C.c_double),
                ("cfl", C.c_double), ("sigma", C.c_double * 3), ("rho", C.c_double * 3),
                ("r", C.c_double), ("w", C.c_double * 3), ("strike", C.c_double)]


class pr3_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("fine_steps", C.c_int32), ("coarse_steps", C.c_int32),
                ("pad_", C.c_int32), ("last_increment", C.c_double),
                ("increments", C.c_double * (PR_MAX_SLICES + 1)), ("t_fine_ms", C.c_double),
                ("t_coarse_ms", C.c_double), ("t_total_ms", C.c_double),
                ("fine_point_steps", C.c_int64)]


SIGNATURES = [
    ("parareal_plan", C.c_int, [C.POINTER(pr_grid), C.POINTER(pr_model), C.POINTER(pr_options),
                                C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("parareal_workspace_bytes", C.c_uint64, [C.POINTER(pr_grid), C.POINTER(pr_options)]),
    ("parareal_create", C.c_int, [C.POINTER(pr_grid), C.POINTER(pr_model), C.POINTER(pr_payoff),
                                  C.POINTER(pr_options), C.c_void_p, C.c_uint64, C.c_void_p,
                                  C.POINTER(C.c_void_p)]),
    ("parareal_solve", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(pr_stats)]),
    ("parareal_serial_fine", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(pr_stats)]),
    ("parareal_apply", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    ("parareal_destroy", C.c_int, [C.c_void_p]),
    ("parareal_solve_static", C.c_int, [C.POINTER(pr_grid), C.POINTER(pr_model),
                                        C.POINTER(pr_payoff), C.POINTER(pr_options), C.c_void_p,
                                        C.c_void_p, C.POINTER(pr_stats)]),
    ("parareal_attach_fno", C.c_int, [C.c_void_p, C.c_void_p]),
    ("parareal_fno_pair", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                     C.c_void_p]),
    ("parareal_fno_pairs", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    ("parareal_strerror", C.c_char_p, [C.c_int]),
    ("parareal_last_error", C.c_char_p, [C.c_void_p]),
    ("parareal_abi_version", C.c_int32, []),
    ("pr_server_footprint", C.c_uint64, [C.POINTER(pr_grid), C.POINTER(pr_options)]),
    ("pr_server_create", C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(pr_server_options),
                                   C.POINTER(C.c_void_p)]),
    ("pr_server_submit", C.c_int, [C.c_void_p, C.POINTER(pr_grid), C.POINTER(pr_model),
                                   C.POINTER(pr_payoff), C.POINTER(pr_options), C.c_void_p,
                                   C.POINTER(C.c_int64)]),
    ("pr_server_progress", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)]),
    ("pr_server_poll", C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int32),
                                 C.POINTER(pr_request_info)]),
    ("pr_server_peaks", C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_uint64)]),
    ("pr_server_rejected", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("pr_server_ragged_stats", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64)]),
    ("pr_server_attach_fno", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pr_server_destroy", C.c_int, [C.c_void_p]),
    ("pr_fno_param_count", C.c_uint64, []),
    ("pr_fno_workspace_bytes", C.c_uint64, [C.c_int32]),
    ("pr_fno_create", C.c_int, [C.POINTER(pr_fno_config), C.c_void_p, C.c_uint64, C.c_void_p,
                                C.POINTER(C.c_void_p)]),
    ("pr_fno_set_params", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pr_fno_get_params", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pr_fno_get_grads", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pr_fno_forward", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                 C.c_void_p]),
    ("pr_fno_backward", C.c_int, [C.c_void_p, C.c_void_p]),
    ("pr_fno_loss", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                              C.c_double, C.c_double, C.c_double, C.c_void_p,
                              C.POINTER(C.c_double)]),
    ("pr_fno_adam", C.c_int, [C.c_void_p, C.c_double, C.c_int32]),
    ("pr_fno_train_step", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                    C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32,
                                    C.c_int32, C.POINTER(C.c_double)]),
    ("pr_fno_save", C.c_int, [C.c_void_p, C.c_char_p, C.c_uint64]),
    ("pr_fno_check_file", C.c_int, [C.c_char_p, C.POINTER(pr_fno_file_info)]),
    ("pr_fno_load", C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(pr_fno_file_info)]),
    ("pr_fno_destroy", C.c_int, [C.c_void_p]),
    ("pr_fno_last_error", C.c_char_p, [C.c_void_p]),
    ("pr3_plan", C.c_int, [C.POINTER(pr3_problem), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("pr3_workspace_bytes", C.c_uint64, [C.POINTER(pr3_problem)]),
    ("pr3_create", C.c_int, [C.POINTER(pr3_problem), C.c_void_p, C.c_uint64, C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    ("pr3_solve", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(pr3_stats)]),
    ("pr3_serial_fine", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(pr3_stats)]),
    ("pr3_fine_sweep_probe", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("pr3_destroy", C.c_int, [C.c_void_p]),
    ("pr3_last_error", C.c_char_p, [C.c_void_p]),
]

_lib = None


def lib():
    """Load libparareal.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2404_02521_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class PararealError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def check(status: int, what: str, solver=None) -> None:
    if status != PR_OK:
        detail = lib().parareal_strerror(status).decode()
        if solver:
            extra = lib().parareal_last_error(solver)
            if extra:
                detail += ": " + extra.decode()
        raise PararealError(status, f"{what}: {detail}")
