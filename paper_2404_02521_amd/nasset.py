"""Three-asset Parareal (include/parareal3.h): argument marshalling only.

torch provides the workspace, the output arrays and the stream; every step of
the path runs in libparareal.so (csrc/nasset.hip).
"""
from __future__ import annotations

import ctypes as C

from . import _lib as L


def make_problem(inst) -> L.pr3_problem:
    p = L.pr3_problem()
    p.n, p.coarse_n, p.n_slices = inst.M, inst.coarse_M, inst.n_slices
    p.max_iters, p.fine_steps, p.coarse_steps = inst.max_iters, inst.fine_steps, inst.coarse_steps
    p.s_max, p.T, p.tol, p.cfl = inst.s_max, inst.T, inst.tol, inst.cfl
    p.sigma[:] = list(inst.sigma)
    p.rho[:] = list(inst.rho)
    p.r = inst.r
    p.w[:] = list(inst.w)
    p.strike = inst.strike
    return p


def plan(inst):
    """(fine steps, coarse steps) per slice."""
    p = make_problem(inst)
    mf, mg = C.c_int32(), C.c_int32()
    L.check(L.lib().pr3_plan(C.byref(p), C.byref(mf), C.byref(mg)), "pr3_plan")
    return mf.value, mg.value


def _stats(st: L.pr3_stats) -> dict:
    return dict(iters=st.iters, fine_steps=st.fine_steps, coarse_steps=st.coarse_steps,
                last_increment=st.last_increment,
                increments=[st.increments[k] for k in range(st.iters)],
                t_fine_ms=st.t_fine_ms, t_coarse_ms=st.t_coarse_ms, t_total_ms=st.t_total_ms,
                fine_point_steps=st.fine_point_steps)


class Solver3:
    def __init__(self, inst, device=None, stream=None):
        import torch
        self.inst = inst
        self.device = torch.device(device or "cuda")
        self._p = make_problem(inst)
        nbytes = int(L.lib().pr3_workspace_bytes(C.byref(self._p)))
        if nbytes == 0:
            raise L.PararealError(L.PR_EINVAL, "pr3_workspace_bytes: invalid problem")
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ws.data_ptr() + 255) // 256 * 256
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        L.check(L.lib().pr3_create(C.byref(self._p), C.c_void_p(ptr), C.c_uint64(nbytes),
                                   C.c_void_p(st.cuda_stream), C.byref(h)), "pr3_create")
        self._h = h

    def _out(self):
        import torch
        n = self.inst.M
        return torch.empty((n, n, n), dtype=torch.float64, device=self.device)

    def _run(self, fn, what):
        out = self._out()
        st = L.pr3_stats()
        rc = fn(self._h, C.c_void_p(out.data_ptr()), C.byref(st))
        if rc not in (L.PR_OK, L.PR_ENOTCONV):
            msg = L.lib().pr3_last_error(self._h).decode()
            raise L.PararealError(rc, f"{what}: {L.lib().parareal_strerror(rc).decode()} {msg}")
        d = _stats(st)
        d["status"] = rc
        return out, d

    def solve(self):
        """(V at tau = T on the full n^3 grid, stats)."""
        return self._run(L.lib().pr3_solve, "pr3_solve")

    def serial_fine(self):
        return self._run(L.lib().pr3_serial_fine, "pr3_serial_fine")

    def sweep_probe(self):
        """(GPU ms of one fine sweep over every slice, interior point-steps)."""
        ms, ps = C.c_double(), C.c_int64()
        L.check(L.lib().pr3_fine_sweep_probe(self._h, C.byref(ms), C.byref(ps)),
                "pr3_fine_sweep_probe")
        return ms.value, ps.value

    def close(self):
        if getattr(self, "_h", None):
            L.lib().pr3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
