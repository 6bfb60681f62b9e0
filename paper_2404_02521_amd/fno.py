"""Fourier neural operator of ``include/parareal.h`` (``pr_fno_*``): ctypes marshalling.

Every computation (forward, backward, loss, Adam) runs in the HIP library;
torch provides the workspace, the tensors and the stream.
"""
from __future__ import annotations

import ctypes as C
import os

from . import _lib as L

GRID = L.PR_FNO_GRID


def _check(st: int, what: str, handle=None) -> None:
    if st != L.PR_OK:
        msg = L.lib().parareal_strerror(st).decode()
        if handle:
            extra = L.lib().pr_fno_last_error(handle)
            if extra:
                msg += ": " + extra.decode()
        raise L.PararealError(st, f"{what}: {msg}")


def param_count() -> int:
    return int(L.lib().pr_fno_param_count())


def _info_dict(info) -> dict:
    return dict(version=info.version, base=info.base, precision=info.precision,
                out_scale=info.out_scale, param_count=info.param_count,
                train_hash=info.train_hash)


def check_file(path: str) -> dict:
    """Validate a weight file on the host (no GPU); raises PararealError(PR_EMODEL)
    for a missing, truncated, corrupted or incompatible file."""
    info = L.pr_fno_file_info()
    _check(L.lib().pr_fno_check_file(os.fsencode(path), C.byref(info)), "pr_fno_check_file")
    return _info_dict(info)


def _ptr(t, dtype, shape=None):
    import torch
    assert t.is_cuda and t.dtype == dtype and t.is_contiguous(), (t.device, t.dtype)
    if shape is not None:
        assert tuple(t.shape) == tuple(shape), (tuple(t.shape), shape)
    return C.c_void_p(t.data_ptr())


class Fno:
    """One FNO handle with its workspace (parameters, gradients, Adam moments and
    the activations of up to ``max_batch`` samples)."""

    def __init__(self, max_batch: int = 1, precision: int = L.PR_FNO_FP32,
                 out_scale: float = 1.0, base: int = L.PR_FNO_BASE_IDENTITY, device=None,
                 stream=None):
        import torch
        self.device = torch.device(device or "cuda")
        self.stream = stream or torch.cuda.current_stream(self.device)
        lib = L.lib()
        nbytes = int(lib.pr_fno_workspace_bytes(max_batch))
        if nbytes == 0:
            raise L.PararealError(L.PR_EINVAL, f"max_batch {max_batch} out of range")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        cfg = L.pr_fno_config(max_batch, precision, out_scale, base, 0)
        h = C.c_void_p()
        _check(lib.pr_fno_create(C.byref(cfg), C.c_void_p(self.ws.data_ptr()), nbytes,
                                 C.c_void_p(self.stream.cuda_stream), C.byref(h)), "pr_fno_create")
        self.handle = h
        self.max_batch = max_batch
        self.out_scale = out_scale
        self.base = base
        self.n_params = param_count()

    # -- parameters ---------------------------------------------------------
    def set_params(self, flat) -> None:
        import torch
        flat = flat.to(device=self.device, dtype=torch.float32).contiguous()
        _check(L.lib().pr_fno_set_params(self.handle, _ptr(flat, torch.float32, (self.n_params,))),
               "pr_fno_set_params", self.handle)
        self.stream.synchronize()

    def params(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(L.lib().pr_fno_get_params(self.handle, _ptr(out, torch.float32)),
               "pr_fno_get_params", self.handle)
        self.stream.synchronize()
        return out

    def grads(self):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(L.lib().pr_fno_get_grads(self.handle, _ptr(out, torch.float32)),
               "pr_fno_get_grads", self.handle)
        self.stream.synchronize()
        return out

    # -- weight files -----------------------------------------------------------
    def save(self, path: str, train_hash: int = 0) -> None:
        """Write the FP32 master weights with the header of pr_fno_save."""
        _check(L.lib().pr_fno_save(self.handle, os.fsencode(path), C.c_uint64(train_hash)),
               "pr_fno_save", self.handle)

    def load(self, path: str) -> dict:
        """Read weights written by save (validated first); returns the file's header."""
        info = L.pr_fno_file_info()
        _check(L.lib().pr_fno_load(self.handle, os.fsencode(path), C.byref(info)),
               "pr_fno_load", self.handle)
        return _info_dict(info)

    # -- compute --------------------------------------------------------------
    def forward(self, w, meta, precision: int = L.PR_FNO_FP32):
        import torch
        B = w.shape[0]
        out = torch.empty((B, GRID, GRID), dtype=torch.float32, device=self.device)
        _check(L.lib().pr_fno_forward(self.handle, _ptr(w, torch.float32, (B, GRID, GRID)),
                                      _ptr(meta, torch.float32, (B, 4)), B, precision,
                                      _ptr(out, torch.float32)), "pr_fno_forward", self.handle)
        self.stream.synchronize()
        return out

    def backward(self, gout) -> None:
        import torch
        _check(L.lib().pr_fno_backward(self.handle, _ptr(gout, torch.float32)),
               "pr_fno_backward", self.handle)
        self.stream.synchronize()

    def loss(self, pred, pairs, meta, dT: float, lam: float = 1.0, scale: float = 1.0):
        """Returns ((loss, data, residual), dLoss/dpred)."""
        import torch
        B = pred.shape[0]
        g = torch.empty((B, GRID, GRID), dtype=torch.float32, device=self.device)
        res = (C.c_double * 3)()
        _check(L.lib().pr_fno_loss(self.handle, _ptr(pred, torch.float32, (B, GRID, GRID)),
                                   _ptr(pairs, torch.float32, (B, 4, GRID, GRID)),
                                   _ptr(meta, torch.float32, (B, 4)), B, scale, dT, lam,
                                   _ptr(g, torch.float32), res), "pr_fno_loss", self.handle)
        return (res[0], res[1], res[2]), g

    def adam(self, lr: float, step: int) -> None:
        _check(L.lib().pr_fno_adam(self.handle, lr, step), "pr_fno_adam", self.handle)
        self.stream.synchronize()

    def train_step(self, pairs, meta, idx, dT: float, lr: float, step: int,
                   precision: int = L.PR_FNO_BF16, lam: float = 1.0, want_loss: bool = True):
        import torch
        B = idx.shape[0]
        res = (C.c_double * 3)()
        assert pairs.shape[0] == meta.shape[0], (pairs.shape, meta.shape)
        _check(L.lib().pr_fno_train_step(self.handle, _ptr(pairs, torch.float32),
                                         _ptr(meta, torch.float32), pairs.shape[0],
                                         _ptr(idx, torch.int32), B, dT, lam, lr, step, precision,
                                         res if want_loss else None),
               "pr_fno_train_step", self.handle)
        return (res[0], res[1], res[2]) if want_loss else None

    def close(self) -> None:
        if getattr(self, "handle", None):
            L.lib().pr_fno_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
