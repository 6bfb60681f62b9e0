"""Write the FP64 oracle's serial fine solutions of the bench workloads to
tests/golden/ (calls only oracle/; the inputs come from synthetic/).

* ``c2_serial_f_seed<s>.npy`` (s = 0..7): the 513 x 513 at-scale problem of
  seed s (N = 64, T = 1, explicit steps at 0.9 of the Gershgorin bound), serial
  F at tau = T on every 4th node (129 x 129, nodes 0, 4, ..., 512).
* ``c5_serial_f_257.npy``: the 2049 x 2049 single solve (N = 256, T = 2), serial
  F on every 8th node (257 x 257).  About 7.7e12 point-steps, hours on a few
  cores; the run checkpoints the state after every slice in --ckpt and resumes
  from the last one.
* ``paper_serial_f_301.npy`` and ``paper_serial_g_301.npy``: the paper's
  cash-or-nothing problem (Sec. 3.2) on its 301 x 301 grid, closed-form ring,
  implicit Euler over N = 10 slices of 0.1: serial F (three steps of 1/30 per
  slice) and the coarse propagator alone (one step of 0.1 per slice), every node;
  their relative l2 errors against the closed form go into the JSON.
* ``bench_oracle.json``: the parameters, step counts and subsample of every file.

Serial F is Eq. (fd)'s spatial operator with explicit Euler (Sec. 3.2) over
the slices of Sec. 3.1 in order; the slice-by-slice loop below performs the
same calls as the oracle's own serial driver (F over slice n from tau = n dT).
Run from the repository root:

    python tests/golden/make_bench_oracle.py --c2
    python tests/golden/make_bench_oracle.py --c5 --ckpt /tmp/c5_ckpt
    python tests/golden/make_bench_oracle.py --paper
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import cash  # noqa: E402
from oracle import implicit  # noqa: E402
from synthetic import largest_single, paper_benchmark, plain_at_scale  # noqa: E402


def problem(inst):
    return oracle.Problem(M=inst.M, sigma1=inst.sigma1, sigma2=inst.sigma2, rho=inst.rho,
                          r=inst.r, payoff_kind=inst.payoff, w1=inst.w1, w2=inst.w2,
                          strike=inst.strike, s_max=inst.s_max)


def serial_f(inst, ckpt=None, log=None):
    p = problem(inst)
    N, T = inst.n_slices, inst.T
    dT = T / N
    mF = oracle.steps_for(p, dT, inst.cfl)
    u, n0 = oracle.payoff_grid(p), 0
    if ckpt:
        os.makedirs(ckpt, exist_ok=True)
        done = sorted(int(f[6:-4]) for f in os.listdir(ckpt)
                      if f.startswith("slice_") and f.endswith(".npy"))
        if done:
            n0 = done[-1]
            u = np.load(os.path.join(ckpt, "slice_%04d.npy" % n0))
    t0 = time.time()
    for n in range(n0, N):
        u = oracle.fine(p, mF, dT / mF, n * dT, u)
        if ckpt:
            np.save(os.path.join(ckpt, "slice_%04d.npy" % (n + 1)), u)
            prev = os.path.join(ckpt, "slice_%04d.npy" % n)
            if n > 0 and os.path.exists(prev):
                os.remove(prev)
        if log:
            log("slice %d/%d done (%.0f s)" % (n + 1, N, time.time() - t0))
    return u, mF


def record(meta, name, inst, mF, every, arr):
    meta[name] = dict(M=inst.M, n_slices=inst.n_slices, T=inst.T, cfl=inst.cfl,
                      fine_steps_per_slice=mF, sigma1=inst.sigma1, sigma2=inst.sigma2,
                      rho=inst.rho, r=inst.r, w1=inst.w1, w2=inst.w2, strike=inst.strike,
                      every=every, shape=list(arr.shape),
                      sha256=hashlib.sha256(arr.tobytes()).hexdigest())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--c2", action="store_true")
    ap.add_argument("--c5", action="store_true")
    ap.add_argument("--seeds", type=int, nargs="*", default=list(range(8)))
    ap.add_argument("--paper", action="store_true")
    ap.add_argument("--ckpt", default=None, help="checkpoint directory of the 2049^2 run")
    args = ap.parse_args()
    mpath = os.path.join(HERE, "bench_oracle.json")
    meta = json.load(open(mpath)) if os.path.exists(mpath) else {}
    log = lambda m: print(m, flush=True)
    if args.c2:
        for s in args.seeds:
            inst = plain_at_scale(s)
            t = time.time()
            u, mF = serial_f(inst)
            sub = np.ascontiguousarray(u[::4, ::4])
            name = "c2_serial_f_seed%d.npy" % s
            np.save(os.path.join(HERE, name), sub)
            record(meta, name, inst, mF, 4, sub)
            log("%s: %d steps per slice, %.1f s" % (name, mF, time.time() - t))
            json.dump(meta, open(mpath, "w"), indent=1, sort_keys=True)
    if args.c5:
        inst = largest_single()
        u, mF = serial_f(inst, ckpt=args.ckpt, log=log)
        sub = np.ascontiguousarray(u[::8, ::8])
        name = "c5_serial_f_257.npy"
        np.save(os.path.join(HERE, name), sub)
        record(meta, name, inst, mF, 8, sub)
        json.dump(meta, open(mpath, "w"), indent=1, sort_keys=True)
        log("%s written" % name)
    if args.paper:
        inst = paper_benchmark()
        p = cash.CashProblem(M=inst.M, s_max=inst.s_max, sigma1=inst.sigma1,
                             sigma2=inst.sigma2, rho=inst.rho, r=inst.r, K1=inst.strike,
                             K2=inst.strike2, cash=inst.cash)
        ex = cash.exact_grid(p, inst.T)
        for tag, m in (("f", inst.fine_steps_per_slice), ("g", inst.coarse_steps_per_slice)):
            t = time.time()
            u = implicit.serial_fine(p, inst.n_slices, inst.T, m, ring=cash.ring_grid,
                                     init=cash.payoff_grid)
            name = "paper_serial_%s_301.npy" % tag
            np.save(os.path.join(HERE, name), u)
            meta[name] = dict(M=inst.M, n_slices=inst.n_slices, T=inst.T, steps_per_slice=m,
                              sigma1=inst.sigma1, sigma2=inst.sigma2, rho=inst.rho, r=inst.r,
                              K1=inst.strike, K2=inst.strike2, cash=inst.cash, every=1,
                              shape=list(u.shape), rel_l2_vs_closed_form=cash.rel_l2(u, ex),
                              sha256=hashlib.sha256(u.tobytes()).hexdigest())
            log("%s: rel l2 vs closed form %.4e, %.1f s" % (name, cash.rel_l2(u, ex),
                                                            time.time() - t))
        json.dump(meta, open(mpath, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
