"""Serving front end: continuous batching of Parareal solves (pr_server_* C ABI).

torch provides the device arena and the output tensors; admission, stream
assignment, iteration scheduling and retirement run in the library's C++
scheduler.  ``run_poisson`` replays a Poisson arrival trace against a server
and reports latency percentiles (nearest rank, host clock from each request's
scheduled arrival to the observed completion) and throughput.
"""
from __future__ import annotations

import ctypes as C
import math
import time

from . import _lib as L
from .parareal import make_structs


class Server:
    def __init__(self, arena_bytes: int, max_resident: int = 64, n_streams: int = 4,
                 device=None, max_queued: int = 0, ragged: bool = False):
        """ragged: PR_SERVER_RAGGED_F (the fine sweeps of the requests ready in a
        progress pass share step launches)."""
        import torch
        self.device = torch.device(device or "cuda")
        self._arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._arena.data_ptr() + 255) // 256 * 256
        o = L.pr_server_options(max_resident, n_streams,
                                L.PR_SERVER_RAGGED_F if ragged else 0, max_queued)
        h = C.c_void_p()
        L.check(L.lib().pr_server_create(C.c_void_p(ptr), C.c_uint64(int(arena_bytes)),
                                         C.byref(o), C.byref(h)), "pr_server_create")
        self._h = h
        self._out = {}
        self._fno = None

    @staticmethod
    def footprint(inst, coarse_kind=L.PR_G_LOD) -> int:
        g, _, _, o = make_structs(inst, coarse_kind)
        return int(L.lib().pr_server_footprint(C.byref(g), C.byref(o)))

    def attach_fno(self, fno) -> None:
        """The operator of PR_G_FNO requests (a paper_2404_02521_amd.fno.Fno, kept
        alive by the server); None clears it."""
        L.check(L.lib().pr_server_attach_fno(self._h, fno.handle if fno is not None else None),
                "pr_server_attach_fno")
        self._fno = fno

    def submit(self, inst, coarse_kind: int = L.PR_G_LOD, max_iters: int = 0,
               bc_kind: int = L.PR_BC_FORWARD_INTRINSIC, flags: int = 0):
        """Queue a solve; returns its id, or None when the bounded queue refused
        it (PR_EBUSY)."""
        import torch
        g, m, p, o = make_structs(inst, coarse_kind, max_iters, bc_kind, flags)
        out = torch.empty((inst.M, inst.M), dtype=torch.float64, device=self.device)
        rid = C.c_int64()
        st = L.lib().pr_server_submit(self._h, C.byref(g), C.byref(m), C.byref(p), C.byref(o),
                                      C.c_void_p(out.data_ptr()), C.byref(rid))
        if st == L.PR_EBUSY:
            return None
        L.check(st, "pr_server_submit")
        self._out[rid.value] = out
        return rid.value

    def rejected(self) -> int:
        n = C.c_int64()
        L.check(L.lib().pr_server_rejected(self._h, C.byref(n)), "pr_server_rejected")
        return n.value

    def ragged_stats(self) -> dict:
        """Progress passes with shared fine sweeps, shared step launches, and the
        request entries they carried."""
        t, n, e = C.c_int64(), C.c_int64(), C.c_int64()
        L.check(L.lib().pr_server_ragged_stats(self._h, C.byref(t), C.byref(n), C.byref(e)),
                "pr_server_ragged_stats")
        return {"ticks": t.value, "launches": n.value, "entries": e.value}

    def progress(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(L.lib().pr_server_progress(self._h, C.byref(a), C.byref(b), C.byref(c)),
                "pr_server_progress")
        return a.value, b.value, c.value

    def poll(self, rid: int):
        done = C.c_int32()
        info = L.pr_request_info()
        L.check(L.lib().pr_server_poll(self._h, rid, C.byref(done), C.byref(info)),
                "pr_server_poll")
        if not done.value:
            return None
        return dict(status=info.status, iters=info.iters, last_increment=info.last_increment,
                    latency_ms=info.latency_ms, queue_ms=info.queue_ms,
                    workspace_bytes=info.workspace_bytes, coarse_fallback=info.coarse_fallback)

    def result(self, rid: int):
        return self._out[rid]

    def release(self, rid: int):
        self._out.pop(rid, None)

    def peaks(self):
        a, b = C.c_int32(), C.c_uint64()
        L.check(L.lib().pr_server_peaks(self._h, C.byref(a), C.byref(b)), "pr_server_peaks")
        return a.value, b.value

    def drain(self, ids, timeout_s: float = 600.0):
        """Run the scheduler until every id in `ids` is done; returns {id: info}."""
        left = set(ids)
        infos = {}
        t0 = time.perf_counter()
        while left:
            self.progress()
            for rid in list(left):
                info = self.poll(rid)
                if info is not None:
                    infos[rid] = info
                    left.discard(rid)
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"{len(left)} requests still running")
        return infos

    def close(self):
        if getattr(self, "_h", None):
            L.lib().pr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def nearest_rank(xs, p):
    xs = sorted(xs)
    return xs[max(1, math.ceil(p / 100.0 * len(xs))) - 1]


def run_poisson(server: Server, arrivals, instances, coarse_kind: int = L.PR_G_LOD,
                timeout_s: float = 600.0, keep_results: bool = False):
    """Submit instances[i] at wall time arrivals[i] (seconds from start), run the
    scheduler, and return latency and throughput figures."""
    n = len(instances)
    ids = [None] * n
    done_t = [None] * n
    infos = [None] * n
    nxt = 0
    pending = {}
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= now:
            rid = server.submit(instances[nxt], coarse_kind)
            ids[nxt] = rid
            if rid is not None:   # None: refused by the bounded queue
                pending[rid] = nxt
            nxt += 1
        server.progress()
        for rid in list(pending):
            info = server.poll(rid)
            if info is not None:
                i = pending.pop(rid)
                done_t[i] = time.perf_counter() - t0
                infos[i] = info
                if not keep_results:
                    server.release(rid)
        if nxt == n and not pending:
            break
        if now > timeout_s:
            raise TimeoutError("Poisson run did not drain")
        if not pending and nxt < n:
            time.sleep(max(0.0, min(0.001, arrivals[nxt] - (time.perf_counter() - t0))))
    served = [i for i in range(n) if ids[i] is not None]
    if not served:
        return dict(count=n, served=0, rejected=n, solves_per_s=0.0, ids=ids)
    lat = [(done_t[i] - arrivals[i]) * 1e3 for i in served]
    span = max(done_t[i] for i in served) - arrivals[0]
    return dict(count=n, served=len(served), rejected=n - len(served),
                solves_per_s=len(served) / span, p50_ms=nearest_rank(lat, 50),
                p99_ms=nearest_rank(lat, 99), mean_ms=sum(lat) / len(lat), span_s=span,
                iters=[infos[i]["iters"] for i in served],
                statuses=[infos[i]["status"] for i in served],
                peak_resident=server.peaks()[0], peak_arena_bytes=server.peaks()[1],
                ids=ids)
