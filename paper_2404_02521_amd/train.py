"""Training the neural coarse propagator on trajectories of the fine propagator.

Data: serial F (the GPU's own explicit propagator) from the payoff over N
slices of a seeded instance; every slice gives one pair restricted to the
64 x 64 operator grid (``parareal_fno_pairs``).  Training: Adam with the step
decay of Sec. 3.5 (lr0 * 0.96 every 25 epochs) on data MSE + PDE residual,
one ``pr_fno_train_step`` per batch.  This module only orders the calls:
shuffling indices, the learning-rate schedule and bookkeeping; every
arithmetic step runs in the HIP library.
"""
from __future__ import annotations

import time

from . import _lib as L


# parameter blocks of the flat vector (include/parareal.h): name, shape, fan-in
def _blocks():
    b = [("L1", (7, 64), 7), ("l1", (64,), 7), ("L2", (64, 32), 64), ("l2", (32,), 64)]
    for l in range(4):
        b += [(f"Rr{l}", (24, 12, 32, 32), 0), (f"Ri{l}", (24, 12, 32, 32), 0),
              (f"W{l}", (32, 32), 32), (f"b{l}", (32,), 32)]
    b += [("P1", (32, 128), 32), ("p1", (128,), 32), ("P2", (128, 1), 128), ("p2", (1,), 128)]
    return b


def init_params(seed: int = 0):
    """Initial flat FP32 parameter vector: dense weights and biases uniform in
    +-1/sqrt(fan_in), spectral multipliers uniform in [0, 1/32^2) (real and
    imaginary parts), drawn block by block in vector order."""
    import numpy as np
    import torch
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape, fan in _blocks():
        if fan == 0:
            parts.append(rng.uniform(0.0, 1.0, size=shape).ravel() / (32 * 32))
        else:
            bound = 1.0 / np.sqrt(fan)
            parts.append(rng.uniform(-bound, bound, size=shape).ravel())
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == int(L.lib().pr_fno_param_count())
    return torch.from_numpy(flat)


def lr_at(epoch: int, lr0: float = 1e-3, decay: float = 0.96, every: int = 25) -> float:
    return lr0 * decay ** (epoch // every)


def generate_pairs(insts, base: int = L.PR_FNO_BASE_IDENTITY, device=None):
    """Stack the pairs of every instance: (P, 4, 64, 64) float32 and meta (P, 4)
    float32 = (sigma1, sigma2, rho, r) of the pair's instance."""
    import torch
    from .parareal import Solver
    dev = torch.device(device or "cuda")
    total = sum(i.n_slices for i in insts)
    pairs = torch.empty((total, 4, 64, 64), dtype=torch.float32, device=dev)
    meta = torch.empty((total, 4), dtype=torch.float32)
    o = 0
    for inst in insts:
        s = Solver(inst, coarse_kind=L.PR_G_FNO, device=dev)
        n = inst.n_slices
        s.fno_pairs(base, pairs[o:o + n])
        meta[o:o + n] = torch.tensor([inst.sigma1, inst.sigma2, inst.rho, inst.r])
        s.close()
        o += n
    return pairs, meta.to(dev)


def evaluate(net, pairs, meta, dT: float, lam: float = 1.0, batch: int = 64,
             precision: int = L.PR_FNO_FP32):
    """Mean (loss, data, residual) over all pairs, prediction scaled by the
    operator's out_scale; the batches are weighted by their size."""
    P = pairs.shape[0]
    acc = [0.0, 0.0, 0.0]
    for b0 in range(0, P, batch):
        pb = pairs[b0:b0 + batch]
        mb = meta[b0:b0 + batch].contiguous()
        out = net.forward(pb[:, 0].contiguous(), mb, precision)
        (lo, da, re), _ = net.loss(out, pb.contiguous(), mb, dT, lam, net.out_scale)
        for k, v in enumerate((lo, da, re)):
            acc[k] += v * pb.shape[0]
    return tuple(a / P for a in acc)


def train(net, pairs, meta, dT: float, epochs: int, batch: int = 64,
          precision: int = L.PR_FNO_BF16, lam: float = 1.0, seed: int = 0, lr0: float = 1e-3,
          log_every: int = 0, time_budget_s: float = 0.0):
    """Adam over shuffled batches; returns the history [(epoch, step, loss, data,
    residual, seconds)] of the last batch of each logged epoch."""
    import torch
    P = pairs.shape[0]
    nb = P // batch
    assert nb >= 1, "fewer pairs than one batch"
    g = torch.Generator().manual_seed(seed)
    hist, step = [], 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(P, generator=g)[: nb * batch].to(torch.int32).to(pairs.device)
        lr = lr_at(ep, lr0)
        for b in range(nb):
            step += 1
            last = b == nb - 1 and log_every and (ep % log_every == 0 or ep == epochs - 1)
            res = net.train_step(pairs, meta, perm[b * batch:(b + 1) * batch], dT, lr, step,
                                 precision, lam, want_loss=bool(last))
            if last:
                hist.append((ep, step) + tuple(res) + (time.perf_counter() - t0,))
        if time_budget_s and time.perf_counter() - t0 > time_budget_s:
            break
    torch.cuda.synchronize()
    if not hist or hist[-1][1] != step:   # stopped between logged epochs
        nan = float("nan")
        hist.append((ep, step, nan, nan, nan, time.perf_counter() - t0))
    return hist
