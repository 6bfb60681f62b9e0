"""Python front end of the C ABI: torch supplies device memory and the stream.

Nothing here computes: the workspace and outputs are torch tensors on the
current HIP device, their pointers and the current stream are handed to the
library, and the library runs every step of the method in its own kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

from . import _lib as L


@dataclass
class SolveResult:
    value: "object"            # torch.Tensor (n, n) float64 on the device
    iters: int
    increments: list = field(default_factory=list)
    status: int = 0
    stats: dict = field(default_factory=dict)


def _stats_dict(st: L.pr_stats) -> dict:
    return dict(status=st.status, iters=st.iters, fine_steps=st.fine_steps,
                coarse_steps=st.coarse_steps, last_increment=st.last_increment, scale=st.scale,
                t_total_ms=st.t_total_ms, t_fine_ms=st.t_fine_ms, t_chain_ms=st.t_chain_ms,
                t_correct_ms=st.t_correct_ms, fine_point_steps=st.fine_point_steps,
                fine_step_launches=st.fine_step_launches, fine_step_bytes=st.fine_step_bytes,
                t_step_kernels_ms=st.t_step_kernels_ms, workspace_bytes=st.workspace_bytes,
                coarse_fallback=st.coarse_fallback, timed_step_launches=st.timed_step_launches,
                timed_step_bytes=st.timed_step_bytes, krylov_iters=st.krylov_iters,
                krylov_max_step=st.krylov_max_step, krylov_unconverged=st.krylov_unconverged)


def make_structs(inst, coarse_kind: int = L.PR_G_NUMERICAL, max_iters: int = 0,
                 bc_kind: int = L.PR_BC_FORWARD_INTRINSIC, flags: int = 0):
    """pr_grid / pr_model / pr_payoff / pr_options from a synthetic.Instance."""
    g = L.pr_grid(inst.M, 0, inst.s_max)
    m = L.pr_model(inst.sigma1, inst.sigma2, inst.rho, inst.r, inst.T)
    p = L.pr_payoff(inst.payoff, bc_kind, inst.w1, inst.w2, inst.strike,
                    getattr(inst, "strike2", 0.0), getattr(inst, "cash", 0.0))
    o = L.pr_options(n_slices=inst.n_slices, max_iters=max_iters, tol=inst.tol,
                     tol_relative=int(inst.tol_relative),
                     precision=L.PR_FP32 if inst.fp32 else L.PR_FP64,
                     fine_steps=inst.fine_steps_per_slice, coarse_kind=coarse_kind,
                     coarse_n=inst.coarse_M, coarse_steps=inst.coarse_steps_per_slice,
                     cfl=inst.cfl, flags=flags,
                     fine_scheme=L.PR_FINE_IMPLICIT if getattr(inst, "implicit", False)
                     else L.PR_FINE_EXPLICIT,
                     krylov_tol=getattr(inst, "krylov_tol", 0.0), krylov_max_iters=0, pad2_=0)
    return g, m, p, o


def plan(inst, coarse_kind: int = L.PR_G_NUMERICAL):
    """(fine_steps, coarse_steps, dt_stable_fine, dt_stable_coarse); host only."""
    g, m, _, o = make_structs(inst, coarse_kind)
    mf, mc = C.c_int32(), C.c_int32()
    df, dc = C.c_double(), C.c_double()
    st = L.lib().parareal_plan(C.byref(g), C.byref(m), C.byref(o), C.byref(mf), C.byref(mc),
                               C.byref(df), C.byref(dc))
    L.check(st, "parareal_plan")
    return mf.value, mc.value, df.value, dc.value


def solve_static(inst, coarse_kind: int = L.PR_G_NUMERICAL, max_iters: int = 0,
                 bc_kind: int = L.PR_BC_FORWARD_INTRINSIC, device=None, stream=None,
                 out=None) -> SolveResult:
    """One solve through parareal_solve_static: the library's static device
    scratch is the workspace, so nothing is allocated but the output tensor
    (pass ``out`` to allocate nothing at all)."""
    import torch
    device = torch.device(device or "cuda")
    g, m, p, o = make_structs(inst, coarse_kind, max_iters, bc_kind, 0)
    if out is None:
        out = torch.empty((inst.M, inst.M), dtype=torch.float64, device=device)
    assert out.dtype == torch.float64 and out.is_contiguous() and out.shape == (inst.M, inst.M)
    stream = stream if stream is not None else torch.cuda.current_stream(device)
    st = L.pr_stats()
    status = L.lib().parareal_solve_static(C.byref(g), C.byref(m), C.byref(p), C.byref(o),
                                           C.c_void_p(stream.cuda_stream),
                                           C.c_void_p(out.data_ptr()), C.byref(st))
    if status not in (L.PR_OK, L.PR_ENOTCONV):
        L.check(status, "parareal_solve_static")
    return SolveResult(out, st.iters, list(st.increments[:st.iters]), status, _stats_dict(st))


class Solver:
    """One solver bound to a workspace tensor and the current stream."""

    def __init__(self, inst, coarse_kind: int = L.PR_G_NUMERICAL, max_iters: int = 0,
                 bc_kind: int = L.PR_BC_FORWARD_INTRINSIC, device=None, stream=None,
                 flags: int = 0):
        import torch
        self.inst = inst
        self.device = torch.device(device or "cuda")
        self._structs = make_structs(inst, coarse_kind, max_iters, bc_kind, flags)
        g, m, p, o = self._structs
        nbytes = L.lib().parareal_workspace_bytes(C.byref(g), C.byref(o))
        if nbytes == 0:
            raise L.PararealError(L.PR_EINVAL, "parareal_workspace_bytes: invalid arguments")
        # 256-byte aligned workspace carved from a torch allocation
        self._ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = L.lib().parareal_create(C.byref(g), C.byref(m), C.byref(p), C.byref(o),
                                     C.c_void_p(self._ws_ptr), C.c_uint64(int(nbytes)),
                                     C.c_void_p(self.stream.cuda_stream), C.byref(h))
        L.check(st, "parareal_create")
        self._h = h
        self.workspace_bytes = int(nbytes)

    def _out(self):
        import torch
        return torch.empty((self.inst.M, self.inst.M), dtype=torch.float64, device=self.device)

    def solve(self, out=None, raise_on_notconv: bool = False) -> SolveResult:
        out = self._out() if out is None else out
        st = L.pr_stats()
        status = L.lib().parareal_solve(self._h, C.c_void_p(out.data_ptr()), C.byref(st))
        if status not in (L.PR_OK, L.PR_ENOTCONV) or (raise_on_notconv and status != L.PR_OK):
            L.check(status, "parareal_solve", self._h)
        return SolveResult(out, st.iters, list(st.increments[:st.iters]), status, _stats_dict(st))

    def serial_fine(self, out=None) -> SolveResult:
        out = self._out() if out is None else out
        st = L.pr_stats()
        status = L.lib().parareal_serial_fine(self._h, C.c_void_p(out.data_ptr()), C.byref(st))
        L.check(status, "parareal_serial_fine", self._h)
        return SolveResult(out, 0, [], status, _stats_dict(st))

    def apply(self, op: int, slice_: int, x):
        """F (op=PR_OP_FINE) or G (PR_OP_COARSE) over one slice of a full grid."""
        import torch
        assert x.dtype == torch.float64 and x.is_contiguous() and x.shape == (self.inst.M,) * 2
        out = self._out()
        status = L.lib().parareal_apply(self._h, op, slice_, C.c_void_p(x.data_ptr()),
                                        C.c_void_p(out.data_ptr()))
        L.check(status, "parareal_apply", self._h)
        return out

    def attach_fno(self, fno) -> None:
        """PR_G_FNO: use the operator of a paper_2404_02521_amd.fno.Fno handle as G."""
        L.check(L.lib().parareal_attach_fno(self._h, fno.handle), "parareal_attach_fno", self._h)
        self._fno = fno

    def fno_pair(self, slice_: int, v0, v1, base: int = L.PR_FNO_BASE_IDENTITY, out=None):
        """PR_G_FNO: training pair [w_in, B1, V_in, V_tgt] (4, 64, 64) float32 of slice
        `slice_` from the full fine grids v0 (at its start) and v1 (at its end)."""
        import torch
        for x in (v0, v1):
            assert x.dtype == torch.float64 and x.is_contiguous() and x.shape == (self.inst.M,) * 2
        if out is None:
            out = torch.empty((4, 64, 64), dtype=torch.float32, device=self.device)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == 4 * 64 * 64
        L.check(L.lib().parareal_fno_pair(self._h, slice_, C.c_void_p(v0.data_ptr()),
                                          C.c_void_p(v1.data_ptr()), base,
                                          C.c_void_p(out.data_ptr())),
                "parareal_fno_pair", self._h)
        return out

    def fno_pairs(self, base: int = L.PR_FNO_BASE_IDENTITY, out=None):
        """PR_G_FNO: the N training pairs (N, 4, 64, 64) float32 of the serial-F
        trajectory from the payoff."""
        import torch
        N = self.inst.n_slices
        if out is None:
            out = torch.empty((N, 4, 64, 64), dtype=torch.float32, device=self.device)
        assert out.dtype == torch.float32 and out.is_contiguous() and out.numel() == N * 4 * 64 * 64
        L.check(L.lib().parareal_fno_pairs(self._h, base, C.c_void_p(out.data_ptr())),
                "parareal_fno_pairs", self._h)
        return out

    def close(self):
        if getattr(self, "_h", None):
            L.lib().parareal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
