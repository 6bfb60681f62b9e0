#!/usr/bin/env python3
"""Throughput of Parareal for the two-asset Black-Scholes equation on one MI355X.

Workload (one "step" = one full Parareal solve, all of its rows: payoff, coarse
initial sweep, fine sweeps, coarse chains, corrections, norms): the plain
method at scale -- 513 x 513 grid on [0, 4]^2, FP32 fine propagator with FP64
correction and norm, N = 64 slices, numerical coarse propagator on 129 x 129,
explicit dt at 0.9 of the Gershgorin bound on both grids, basket call with
seed-drawn parameters (sigma ~ U[0.1, 0.5], rho ~ U[-0.8, 0.8], r ~ U[0, 0.1],
weights ~ Dirichlet(1, 1), K ~ U[0.5, 1.5]), T = 1.  Step s solves seed
s mod 8.  Every solve's error against the GPU's serial fine solution is checked
outside the timed region.

Prints ONE JSON line: solves/s (value), per-solve latency p50/p99, the
roofline of the dominant kernel (the FP32 explicit step) from HIP events
around runs of 8 consecutive step launches (every launch of the timed solves),
and the FP64 oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s + p99 latency at err≤1e-5 vs serial F; stencil HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
# FP32 operations of one interior point-step of the increment-form update
# d+ = d + dt (Lb + L d): second differences 3 + 3, four-corner difference 3,
# first differences 1 + 1, five coefficient products and the reaction 6 with 5
# additions, then + Lb, * dt, + d.
FLOPS_PER_POINT_STEP = 25
# MI355X FP32 vector peak as published (it counts packed FP32, two FMAs per lane
# per cycle), and the single-issue figure 256 CUs x 4 SIMDs x 16 lanes x 2 flops
# x 2.4 GHz that applies to code built without packed FP32, as this library is
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_VECTOR_NONPACKED_TFLOPS = 78.6
SEEDS = list(range(8))


KERNEL_SOURCES = ("device.hpp", "step_tb.hpp", "kernels.hip")


def kernel_source_hash() -> str:
    """First 16 hex digits of sha256 over the step kernel's sources (device.hpp,
    step_tb.hpp, then kernels.hip)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2404_02521_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def profile_figures(name):
    """`key: value` figures of a committed rocprofv3 summary under profiles/, or
    {} when the summary is missing or was taken on another kernel source."""
    f = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(f):
        return {}
    txt = open(f).read()
    if "kernel_source_sha256: " + kernel_source_hash() not in txt:
        return {}
    out = {}
    for line in txt.splitlines():
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            try:
                out[k.strip()] = float(v)
            except ValueError:
                pass
    return out


def progress(msg):
    """One progress line on stderr (stdout carries only the JSON result)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def golden_oracle(name):
    """A stored FP64 oracle solution (tests/golden/, written by a script that
    calls only the oracle), or None when it has not been generated."""
    import numpy as np
    f = os.path.join(ROOT, "tests", "golden", name)
    return np.load(f) if os.path.exists(f) else None


def rel_err_sub(value, ref, every):
    """Relative max-norm error of a device grid, subsampled every `every` nodes,
    against a stored oracle subsample."""
    import numpy as np
    v = value.detach().cpu().numpy()[::every, ::every]
    return float(np.abs(v - ref).max() / np.abs(ref).max())


def nearest_rank(xs, p):
    xs = sorted(xs)
    k = max(1, math.ceil(p / 100.0 * len(xs)))
    return xs[k - 1]


def host_cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return platform.processor()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seeds", type=int, default=len(SEEDS))
    ap.add_argument("--max-iters", type=int, default=0,
                    help="cap Parareal iterations (counter runs only; 0 = to convergence)")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the error check against serial F (counter runs only)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this size (counter calibration)")
    ap.add_argument("--no-fno", action="store_true", help="skip the neural coarse propagator leg")
    ap.add_argument("--fno-train-only", action="store_true",
                    help="run only the training part of the neural coarse propagator leg")
    ap.add_argument("--largest-solve", action="store_true",
                    help="run only the 2049^2, 256-slice solve (LOD G) against serial F")
    ap.add_argument("--paper-only", action="store_true",
                    help="run only the paper's cash-or-nothing benchmark leg")
    ap.add_argument("--three-asset-probe", default=None,
                    help="M,N: one three-asset fine sweep over N slices of M^3 (profiling)")
    ap.add_argument("--krylov-probe", action="store_true",
                    help="one serial implicit F of the paper problem (profiling)")
    ap.add_argument("--three-asset-only", action="store_true",
                    help="run only the three-asset leg")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving leg")
    ap.add_argument("--paper-spacings", default="1,0.5",
                    help="grid spacings of the resolution study (1, 0.5, 0.25)")
    ap.add_argument("--no-largest", action="store_true",
                    help="skip the 2049^2, 256-slice solve leg")
    ap.add_argument("--largest-share-only", action="store_true",
                    help="run only the 2049^2 x 32-slice step-kernel leg and print its JSON")
    ap.add_argument("--step-probe", default=None,
                    help="M,N: run only the step-kernel probe on an M^2 grid with N slices")
    ap.add_argument("--fno-train-s", type=float, default=30.0,
                    help="training budget of the neural coarse propagator leg (seconds)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2404_02521_amd as pr
    from synthetic import plain_at_scale

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    def copy_probe():
        # a plain device-to-device copy of known size: the calibration of the
        # FETCH_SIZE / WRITE_SIZE counters in the same process
        if args.copy_probe_mib:
            n = args.copy_probe_mib << 20
            src = torch.ones(n, dtype=torch.uint8, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst

    if args.three_asset_probe:
        copy_probe()
        from paper_2404_02521_amd import nasset
        from synthetic import three_asset
        M, N = (int(x) for x in args.three_asset_probe.split(","))
        sp = nasset.Solver3(three_asset(0, M=M, coarse_M=(M - 1) // 4 + 1, n_slices=N))
        sp.sweep_probe()
        ms, ps = sp.sweep_probe()
        sp.close()
        print(json.dumps({"workload": "three-asset %d^3 x %d slices, one fine sweep" % (M, N),
                          "point_steps": ps, "ms": ms, "point_steps_per_s": ps / (ms * 1e-3),
                          "effective_gbs": ps * 16 / (ms * 1e-3) / 1e9}), flush=True)
        return
    if args.krylov_probe:
        copy_probe()
        from synthetic import paper_benchmark
        sv = pr.Solver(paper_benchmark(), bc_kind=pr.PR_BC_EXACT, coarse_kind=pr.PR_G_IMPLICIT)
        r = sv.serial_fine()
        sv.close()
        print(json.dumps({"workload": "paper problem 301^2, serial implicit F (30 steps)",
                          "krylov_iters": r.stats["krylov_iters"],
                          "ms": r.stats["t_total_ms"]}), flush=True)
        return
    if args.largest_share_only or args.step_probe:
        copy_probe()
        if args.step_probe:
            M, N = (int(x) for x in args.step_probe.split(","))
            print(json.dumps(step_probe(pr, M, N)), flush=True)
        else:
            print(json.dumps(largest_share_leg(pr)), flush=True)
        return
    if args.largest_solve:
        print(json.dumps(largest_solve(pr)), flush=True)
        return
    if args.three_asset_only:
        print(json.dumps(three_asset_leg(pr)), flush=True)
        return
    if args.serving_only:
        print(json.dumps(serving_leg(pr)), flush=True)
        return
    if args.paper_only:
        sp = tuple(float(v) for v in args.paper_spacings.split(","))
        print(json.dumps(paper_leg(pr, sp)), flush=True)
        return
    if args.fno_train_only:
        print(json.dumps(fno_leg(pr, [], [], {}, args.fno_train_s, parareal=False)), flush=True)
        return
    seeds = SEEDS[: args.seeds]
    insts = [plain_at_scale(s) for s in seeds]
    if args.copy_probe_mib:
        n = args.copy_probe_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # solvers (workspaces) are created before the timed region: inputs resident in HBM
    # per-launch HIP events around every explicit step, on the solvers' stream
    solvers = {s: pr.Solver(inst, device=dev, flags=pr.PR_FLAG_TIME_STEPS,
                            max_iters=args.max_iters)
               for s, inst in zip(seeds, insts)}

    # correctness outside the timed region: error vs the GPU serial fine solution
    errs, iters, serial_ms = {s: float("nan") for s in seeds}, {s: 0 for s in seeds}, {s: 0.0 for s in seeds}
    errs_oracle, serial_errs_oracle = {}, {}
    serial_ref = {}
    for s in ([] if args.no_check else seeds):
        sv = solvers[s]
        ser = sv.serial_fine()
        serial_ms[s] = ser.stats["t_total_ms"]
        ser_v = ser.value.clone()
        serial_ref[s] = ser_v
        res = sv.solve()
        iters[s] = res.iters
        errs[s] = float((res.value - ser_v).abs().max() / ser_v.abs().max())
        ref = golden_oracle("c2_serial_f_seed%d.npy" % s)
        if ref is not None:
            errs_oracle[s] = rel_err_sub(res.value, ref, 4)
            serial_errs_oracle[s] = rel_err_sub(ser_v, ref, 4)

    progress("correctness pass done")
    for w in range(args.warmup):
        solvers[seeds[w % len(seeds)]].solve()
    torch.cuda.synchronize()

    lat, steps_ms, steps_bytes, steps_launch, chain_ms, fine_ms, corr_ms = [], 0.0, 0.0, 0, 0.0, 0.0, 0.0
    all_bytes, all_launch = 0.0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        s = seeds[k % len(seeds)]
        a = time.perf_counter()
        res = solvers[s].solve()
        lat.append((time.perf_counter() - a) * 1e3)
        st = res.stats
        steps_ms += st["t_step_kernels_ms"]
        steps_bytes += st["timed_step_bytes"]       # the event-timed sample of step launches
        steps_launch += st["timed_step_launches"]
        all_bytes += st["fine_step_bytes"]
        all_launch += st["fine_step_launches"]
        chain_ms += st["t_chain_ms"]
        fine_ms += st["t_fine_ms"]
        corr_ms += st["t_correct_ms"]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    progress("timed region done: %.2f solves/s" % (args.steps / total))

    value = args.steps / total
    # point-steps of the event-timed step launches (12 B algorithmic per point-step)
    pts_per_s = steps_bytes / 12.0 / (steps_ms * 1e-3) if steps_ms > 0 else 0.0
    achieved_tflops = pts_per_s * FLOPS_PER_POINT_STEP / 1e12
    # the profile of these solves' launches: a sweep of 32 slices at 513^2 (the
    # phased overlap's groups and the late iterations cover 1 to 42 slices)
    head = profile_figures("k_fine_tb_513x513x32_fp32.md")
    share = profile_figures("k_fine_tb_2049x2049x32_fp32.md")
    # the kernel trace of this command (bench.py itself): the step kernel's
    # average duration without the events' dispatch delay
    trace = profile_figures("k_fine_tb_headline_513x513x64_fp32.md")
    avg_launch_us = steps_ms * 1e3 / max(1, steps_launch)
    pts_per_launch = steps_bytes / 12.0 / max(1, steps_launch)
    traffic = (round(head["hbm_bytes_per_point_step"] * pts_per_launch)
               if "hbm_bytes_per_point_step" in head else None)
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "plain method at scale: 513x513 basket call on [0,4]^2, FP32 "
                               "explicit F + FP64 correction, N=64, numerical G 129x129, "
                               "dt 0.9x Gershgorin, seeds %d-%d" % (seeds[0], seeds[-1]),
                   "grid": 513, "slices": 64, "coarse_grid": 129, "seeds": seeds},
        "p50_ms": round(nearest_rank(lat, 50), 3),
        "p99_ms": round(nearest_rank(lat, 99), 3),
        "max_err_vs_serial_f": None if args.no_check else max(errs.values()),
        "max_err_vs_oracle": max(errs_oracle.values()) if errs_oracle else None,
        "serial_f_max_err_vs_oracle": (max(serial_errs_oracle.values())
                                       if serial_errs_oracle else None),
        "oracle_reference": "FP64 oracle serial F of each seed on every 4th node (129^2 of "
                            "513^2), stored by tests/golden/make_bench_oracle.py",
        "iters": [iters[s] for s in seeds],
        "serial_f_ms": [round(serial_ms[s], 2) for s in seeds],
        "parareal_ms": [round(x, 2) for x in lat[: len(seeds)]],
        "phase_ms": {"fine_sweeps": round(fine_ms, 2), "coarse_chain": round(chain_ms, 2),
                     "correction": round(corr_ms, 2), "step_kernels_timed": round(steps_ms, 2)},
        "roofline": {
            "bound": "alu", "achieved": round(achieved_tflops, 3), "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "kernel": "k_fine_tb<MODE_INCR, S=5 for sweeps of <= 16 slices, 6 above> (FP32 "
                      "increment form, S explicit steps per launch "
                      "in registers, neighbour weights with dt folded in)",
            "why_alu": "rocprofv3 SQ counters: the kernel issues VALU instructions at the chip's "
                       "VALU issue rate while its HBM traffic stays well below peak (profiles/)",
            "flops_per_point_step": FLOPS_PER_POINT_STEP,
            "point_steps_per_s": round(pts_per_s, 1),
            "peak_without_packed_fp32_tflops": FP32_VECTOR_NONPACKED_TFLOPS,
            "frac_without_packed_fp32": round(achieved_tflops / FP32_VECTOR_NONPACKED_TFLOPS, 4),
            "effective_gbs": round(pts_per_s * 12.0 / 1e9, 1),
            "valu_instr_per_point_step": head.get("valu_instr_per_point_step"),
            "valu_issue_frac": head.get("valu_issue_frac"),
            "hbm_gbs": (round(head["hbm_bytes_per_point_step"] * pts_per_s / 1e9, 1)
                        if "hbm_bytes_per_point_step" in head else None),
            "hbm_frac": (round(head["hbm_bytes_per_point_step"] * pts_per_s / 1e9 / HBM_PEAK_GBS, 4)
                         if "hbm_bytes_per_point_step" in head else None),
            "above_cache_2049x32": {k: share.get(k) for k in (
                "point_steps_per_s", "hbm_bytes_per_point_step", "hbm_gbs", "hbm_frac",
                "valu_instr_per_point_step", "valu_issue_frac", "achieved_tflops")},
            "kernel_source_sha256": kernel_source_hash(),
            "avg_launch_us": round(avg_launch_us, 3),
            "kernel_trace_avg_launch_us": trace.get("kernel_trace_avg_launch_us"),
            "achieved_with_kernel_trace_duration": (
                round(achieved_tflops * avg_launch_us / trace["kernel_trace_avg_launch_us"], 3)
                if trace.get("kernel_trace_avg_launch_us") else None),
            "point_steps_per_launch": round(pts_per_launch),
            "timed_launches": steps_launch, "all_launches": all_launch},
    }
    if not args.no_check:
        # the same timed solves with the coarse chain after each whole fine sweep
        # (no overlap of chain and sweep): what the overlapped schedule gains
        ser_solvers = {s: pr.Solver(inst, device=dev, max_iters=args.max_iters,
                                    flags=pr.PR_FLAG_SERIAL_CHAIN)
                       for s, inst in zip(seeds, insts)}
        ser_solvers[seeds[0]].solve()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ch = 0.0
        for k in range(args.steps):
            ch += ser_solvers[seeds[k % len(seeds)]].solve().stats["t_chain_ms"]
        torch.cuda.synchronize()
        t_ser = time.perf_counter() - t1
        for sv in ser_solvers.values():
            sv.close()
        out["chain_overlap"] = {
            "overlapped_solves_per_s": round(value, 4),
            "serial_chain_solves_per_s": round(args.steps / t_ser, 4),
            "exposed_chain_ms_per_solve": round(chain_ms / args.steps, 2),
            "serial_chain_ms_per_solve": round(ch / args.steps, 2)}
        progress("serial-chain comparison done")
        out["lod_coarse"] = lod_leg(pr, insts, seeds, serial_ref)
        progress("lod leg done")
        out["serving"] = serving_leg(pr)
        progress("serving leg done")
        out["largest_share"] = largest_share_leg(pr)
        out["above_cache_1025x64"] = step_probe(pr, 1025, 64)
        progress("step-kernel probes done")
        out["graph"] = graph_leg(pr)
        progress("graph leg done")
        out["paper_benchmark"] = paper_leg(pr)
        progress("paper benchmark leg done")
        out["three_asset"] = three_asset_leg(pr)
        progress("three-asset leg done")
        if not args.no_fno:
            out["fno_coarse"] = fno_leg(pr, insts, seeds, serial_ref, args.fno_train_s)
            progress("fno leg done")
        if not args.no_largest:
            out["largest_solve"] = largest_solve(pr)
            progress("largest solve done")
    if args.max_iters:
        out["note"] = "iterations capped at %d (counter run, not a bench line)" % args.max_iters
    if not args.no_cpu_baseline and not args.no_check:
        out["cpu_baseline"] = run_cpu_baseline(insts, iters[seeds[0]])
    print(json.dumps(out), flush=True)


def lod_leg(pr, insts, seeds, serial_ref, coarse_steps=4):
    """Same seeds with the same-grid implicit (LOD) coarse propagator, 4 steps per
    slice: one warm solve, then one timed solve per seed."""
    import torch
    lat, iters, errs = [], [], []
    for s, inst in zip(seeds, insts):
        sv = pr.Solver(inst.replace(coarse_steps_per_slice=coarse_steps), coarse_kind=pr.PR_G_LOD)
        sv.solve()
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = sv.solve()
        lat.append((time.perf_counter() - t) * 1e3)
        iters.append(res.iters)
        ref = serial_ref[s]
        errs.append(float((res.value - ref).abs().max() / ref.abs().max()))
        sv.close()
    return {"workload": "same seeds, same-grid implicit coarse propagator (LOD, %d steps per "
                        "slice) instead of the 129^2 explicit one" % coarse_steps,
            "solves_per_s": round(len(lat) / (sum(lat) * 1e-3), 4),
            "p50_ms": round(nearest_rank(lat, 50), 3), "p99_ms": round(nearest_rank(lat, 99), 3),
            "iters": iters, "max_err_vs_serial_f": max(errs),
            "parareal_ms": [round(x, 2) for x in lat]}


def largest_solve(pr):
    """The largest single solve: 2049^2 FP32, N = 256 slices, T = 2 (7207 explicit
    steps per slice), Parareal with the same-grid implicit G (4 steps per slice)
    against the GPU's serial F (error in the relative max norm), the same with
    every iteration captured as a hipGraph (capture included in the time), then
    two iterations with the numerical G on the 257^2 coarse grid."""
    import torch
    from synthetic import largest_single
    inst = largest_single().replace(coarse_steps_per_slice=4)
    sv = pr.Solver(inst, coarse_kind=pr.PR_G_LOD, flags=pr.PR_FLAG_TIME_STEPS)
    t = time.perf_counter()
    ser = sv.serial_fine()
    torch.cuda.synchronize()
    t_ser = time.perf_counter() - t
    ref = ser.value.clone()
    t = time.perf_counter()
    r = sv.solve()
    torch.cuda.synchronize()
    t_par = time.perf_counter() - t
    err = float((r.value - ref).abs().max() / ref.abs().max())
    st = r.stats
    ora = golden_oracle("c5_serial_f_257.npy")
    ser_err_oracle = None if ora is None else rel_err_sub(ref, ora, 8)
    par_err_oracle = None if ora is None else rel_err_sub(r.value, ora, 8)
    # the same solve with each iteration captured once as a hipGraph and replayed
    sg = pr.Solver(inst, coarse_kind=pr.PR_G_LOD, flags=pr.PR_FLAG_GRAPH)
    t = time.perf_counter()
    rg = sg.solve()
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t
    err_graph = float((rg.value - ref).abs().max() / ref.abs().max())
    iters_graph = rg.iters
    sg.close()
    out = {"workload": "2049^2 FP32 increment form, N=256, T=2, LOD G (4 steps per slice)",
           "workspace_gb": round(sv.workspace_bytes / 2 ** 30, 2),
           "fine_steps_per_slice": st["fine_steps"], "serial_f_s": round(t_ser, 2),
           "parareal_s": round(t_par, 2), "iters": r.iters, "err_vs_serial_f": err,
           "graph_parareal_s": round(t_graph, 2), "graph_iters": iters_graph,
           "graph_err_vs_serial_f": err_graph,
           "serial_f_err_vs_oracle": ser_err_oracle, "parareal_err_vs_oracle": par_err_oracle,
           "oracle_reference": "FP64 oracle serial F at 2049^2 on every 8th node (257^2), "
                               "stored by tests/golden/make_bench_oracle.py",
           "increments": [float("%.3g" % x) for x in r.increments],
           "step_kernel_gbs": round(st["timed_step_bytes"] / (st["t_step_kernels_ms"] * 1e-3) / 1e9, 1),
           "phase_ms": {"fine": round(st["t_fine_ms"], 1),
                        "g_and_corrections": round(st["t_chain_ms"] + st["t_correct_ms"], 1)}}
    sv.close()
    # the specified numerical G (257^2 coarse grid, ratio 8): its chain keeps the
    # coarse state in global memory; two iterations show its per-iteration cost
    # and increments (with this G the iteration does not converge before K = N)
    num = largest_single()
    sn = pr.Solver(num, coarse_kind=pr.PR_G_NUMERICAL, max_iters=2, flags=pr.PR_FLAG_TIME_STEPS)
    t = time.perf_counter()
    rn = sn.solve()
    torch.cuda.synchronize()
    t_num = time.perf_counter() - t
    stn = rn.stats
    out["numerical_g_257"] = {
        "coarse_steps_per_slice": stn["coarse_steps"], "iters_run": rn.iters,
        "wall_s": round(t_num, 2), "increments": [float("%.3g" % x) for x in rn.increments],
        "phase_ms": {"fine": round(stn["t_fine_ms"], 1), "chain": round(stn["t_chain_ms"], 1),
                     "correct": round(stn["t_correct_ms"], 1)}}
    sn.close()
    return out


def paper_leg(pr, fine_spacings=(1.0, 0.5)):
    """The paper's benchmark problem and its experiments (Sec. 3.2, Sec. 4.1,
    Sec. 4.4, Sec. 4.5): the two-asset cash-or-nothing option on [0, 300]^2 with
    the closed form as ring, implicit-Euler F (three steps of 1/30 per slice),
    N = 10 slices, FP64, BiCGStab to 1e-12, with two coarse propagators on the
    same grid and one step of 0.1 per slice: the paper's implicit Euler (a
    BiCGStab solve per step) and the direction-split implicit Euler (LOD: two
    sweeps of tridiagonal line solves per step, no iteration).

    * c_F and c_G per slice (GPU) and the bound of Eq. (speedup) they imply;
    * relative l2 errors of serial F and serial G against the closed form (the
      paper prints 2.2e-3 and 1.0e-2 for its runs, Sec. 4.1), and serial F
      against the stored FP64 oracle;
    * convergence against serial F after each Parareal iteration K (Fig. 3);
    * resolution (Sec. 4.4, with the LOD G): spacing 1 with N = 2, 0.5 with
      N = 4 (and 0.25 with N = 8 when asked for), the time steps halved with
      the grid: 5 coarse and 15 fine steps per slice;
    * parameters (Sec. 4.5, values from its range 0.1 ... 5, with the LOD G): r, sigma1 and
      sigma2 varied one at a time, error per K and the K that reaches 1e-8.

    On one GPU all N slices of a Parareal iteration run in one batched sweep, so
    the measured speedup over serial F is the GPU's (Eq. (speedup) bounds it
    only through the c_G / c_F ratio)."""
    import numpy as np
    import torch
    from synthetic import paper_benchmark

    def rel(a, b):
        return float((a - b).abs().max() / b.abs().max())

    def rel_l2(a, b):
        return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))

    def run(inst, kmax, kind=pr.PR_G_IMPLICIT, timed=()):
        """Serial F (timed on its second call), then Parareal with coarse
        propagator `kind` and max_iters = K for K = 1..kmax: error against
        serial F and last increment per K, and the wall time of the solves whose
        K is in `timed` (second call)."""
        sv = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT, coarse_kind=kind)
        sv.serial_fine()
        torch.cuda.synchronize()
        t = time.perf_counter()
        ser = sv.serial_fine()
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t
        sref = ser.value.clone()
        errs, errs_l2, incs, ms = [], [], [], {}
        for k in range(1, kmax + 1):
            s2 = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT, coarse_kind=kind, max_iters=k)
            r = s2.solve()
            if k in timed:
                torch.cuda.synchronize()
                t = time.perf_counter()
                r = s2.solve()
                torch.cuda.synchronize()
                ms[k] = (time.perf_counter() - t) * 1e3
            errs.append(float("%.3g" % rel(r.value, sref)))
            errs_l2.append(float("%.3g" % rel_l2(r.value, sref)))
            incs.append(float("%.3g" % r.increments[-1]))
            s2.close()
        progress("paper leg: M=%d N=%d r=%g s1=%g s2=%g G=%d done" % (
            inst.M, inst.n_slices, inst.r, inst.sigma1, inst.sigma2, kind))
        return sv, sref, t_f, (errs, errs_l2), incs, ser.stats, ms

    out = {"workload": "cash-or-nothing, [0,300]^2 spacing 1 (301^2), K1=K2=100, r=1, "
                       "sigma=0.3/0.3, rho=0.5, T=1, c=1; implicit F 3 steps/slice, implicit G "
                       "1 step/slice, N=10, FP64, BiCGStab tol 1e-12"}
    inst = paper_benchmark()
    P = inst.n_slices
    x = torch.arange(inst.M, dtype=torch.float64, device="cuda") * (inst.s_max / (inst.M - 1))
    payoff = ((x[:, None] >= inst.strike) & (x[None, :] >= inst.strike2)).double() * inst.cash
    meta = {}
    mp = os.path.join(ROOT, "tests", "golden", "bench_oracle.json")
    if os.path.exists(mp):
        meta = json.load(open(mp))

    def serial_g(kind):
        """The coarse propagator alone, slice by slice from the payoff (second pass timed)."""
        g = pr.Solver(inst, bc_kind=pr.PR_BC_EXACT, coarse_kind=kind, max_iters=1)
        for rep in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            u = payoff
            for n in range(P):
                u = g.apply(pr.PR_OP_COARSE, n, u)
            torch.cuda.synchronize()
            t_g = time.perf_counter() - t
        g.close()
        return u, t_g

    def bound(cg, cf, K):   # Eq. (speedup)
        return 1.0 / ((1.0 + K / P) * cg / cf + K / P)

    t_f = None
    for name, kind in (("implicit", pr.PR_G_IMPLICIT), ("lod", pr.PR_G_LOD)):
        sv, sref, tf, errs, incs, st, ms = run(inst, P, kind, timed=(1, 2))
        if t_f is None:
            t_f = tf
            out["serial_f_ms"] = round(t_f * 1e3, 2)
            out["c_fine_ms_per_slice"] = round(t_f * 1e3 / P, 3)
            out["krylov_iters_per_fine_step"] = round(st["krylov_iters"] / (P * inst.fine_steps_per_slice), 1)
            out["krylov_unconverged"] = st["krylov_unconverged"]
            # stored FP64 oracle solution: max-norm difference, and the oracle's
            # relative l2 error against the closed form (the quantity Sec. 4.1
            # prints: 2.2e-3 for F and 1.0e-2 for G in the paper's runs)
            rl2 = {"paper_printed_f": 2.2e-3, "paper_printed_g": 1.0e-2}
            ref = golden_oracle("paper_serial_f_301.npy")
            if ref is not None and ref.shape == tuple(sref.shape):
                out["serial_f_err_vs_oracle"] = float(np.abs(sref.cpu().numpy() - ref).max())
                rl2["serial_f_oracle"] = meta.get("paper_serial_f_301.npy", {}).get("rel_l2_vs_closed_form")
            out["rel_l2_vs_closed_form"] = rl2
        sv.close()
        ug, t_g = serial_g(kind)
        cf, cg = t_f / P, t_g / P
        row = {"c_coarse_ms_per_slice": round(cg * 1e3, 3),
               "speedup_bound_K1": round(bound(cg, cf, 1), 3),
               "speedup_bound_K2": round(bound(cg, cf, 2), 3),
               "parareal_ms": {str(k): round(v, 2) for k, v in ms.items()},
               "speedup_vs_serial_f": {str(k): round(t_f * 1e3 / v, 3) for k, v in ms.items()},
               "convergence": {"K": list(range(1, P + 1)), "err_vs_serial_f": errs[0],
                               "rel_l2_vs_serial_f": errs[1], "last_increment": incs}}
        if kind == pr.PR_G_IMPLICIT:
            ref = golden_oracle("paper_serial_g_301.npy")
            if ref is not None and ref.shape == tuple(ug.shape):
                row["serial_g_err_vs_oracle"] = float(np.abs(ug.cpu().numpy() - ref).max())
                out["rel_l2_vs_closed_form"]["serial_g_oracle"] = meta.get(
                    "paper_serial_g_301.npy", {}).get("rel_l2_vs_closed_form")
        out["G_" + name] = row
    res = []
    for spacing, N in zip(fine_spacings, (2, 4, 8)):
        ri = paper_benchmark(spacing=spacing, n_slices=N, fine_steps_per_slice=15,
                             coarse_steps_per_slice=5)
        s_, _, tf, e, _, _, _ = run(ri, N, pr.PR_G_LOD)
        s_.close()
        res.append({"spacing": spacing, "grid": ri.M, "N": N, "err_vs_serial_f": e[0],
                    "rel_l2_vs_serial_f": e[1], "serial_f_s": round(tf, 3)})
    out["resolution_lod_g"] = res
    par = []
    for kw in (dict(r=0.1), dict(r=5.0), dict(sigma1=0.1), dict(sigma1=3.0), dict(sigma2=5.0)):
        ri = paper_benchmark(**kw)
        s_, _, _, e, _, _, _ = run(ri, ri.n_slices, pr.PR_G_LOD)
        s_.close()
        k8 = next((k + 1 for k, x in enumerate(e[0]) if x < 1e-8), None)
        par.append(dict(kw, err_vs_serial_f=e[0], rel_l2_vs_serial_f=e[1], K_to_1e_8=k8))
    out["parameters_lod_g"] = par
    # the slice count of the paper's convergence figure (Sec. 4.1): 12 slices of
    # 1/12, one implicit G step and three implicit F steps per slice
    p12 = paper_benchmark(n_slices=12)
    s_, _, _, e, incs12, _, _ = run(p12, 6, pr.PR_G_IMPLICIT)
    s_.close()
    out["convergence_P12_implicit_g"] = {"K": list(range(1, 7)), "err_vs_serial_f": e[0],
                                         "rel_l2_vs_serial_f": e[1], "last_increment": incs12}
    return out


def three_asset_leg(pr):
    """The three-asset generalisation (Eq. (bse_general), n = 3; 19-point
    explicit scheme, FP64): Parareal on 65^3 with N = 16 and G on 17^3 against
    the GPU's serial F, and the step kernel's throughput over all 16 slices at
    65^3 and 129^3 (16 B of HBM per interior point-step: one read, one write;
    49 FP64 operations: 7 for the i-dependent coefficients, 8 per axis, 5 per
    pair, 1 for the reaction, 2 for the update)."""
    import torch
    from paper_2404_02521_amd import nasset
    from synthetic import three_asset
    out = {"workload": "basket call on three assets, seed 0 parameters, [0,4]^3, T=1, N=16, "
                       "explicit F at 0.9 of the Gershgorin bound, G on a 4x coarser grid"}
    inst = three_asset(0, M=65, coarse_M=17, n_slices=16).replace(tol=1e-8)
    s = nasset.Solver3(inst)
    ser, sst = s.serial_fine()
    ser, sst = s.serial_fine()
    torch.cuda.synchronize()
    t = time.perf_counter()
    v, st = s.solve()
    torch.cuda.synchronize()
    t_par = time.perf_counter() - t
    out["65^3_parareal"] = {
        "fine_steps": st["fine_steps"], "coarse_steps": st["coarse_steps"], "iters": st["iters"],
        "err_vs_serial_f": float((v - ser).abs().max() / ser.abs().max()),
        "serial_f_ms": round(sst["t_total_ms"], 2), "parareal_ms": round(t_par * 1e3, 2),
        "increments": [float("%.3g" % x) for x in st["increments"]]}
    s.close()
    for M, Mc in ((65, 17), (129, 33)):
        pi = three_asset(0, M=M, coarse_M=Mc, n_slices=16)
        sp = nasset.Solver3(pi)
        sp.sweep_probe()
        ms, ps = sp.sweep_probe()
        sp.close()
        rate = ps / (ms * 1e-3)
        out["%d^3_sweep" % M] = {"slices": 16, "point_steps": ps, "ms": round(ms, 3),
                                 "point_steps_per_s": round(rate, 1),
                                 "effective_gbs": round(rate * 16 / 1e9, 1),
                                 "hbm_frac_algorithmic": round(rate * 16 / 1e9 / HBM_PEAK_GBS, 4),
                                 "fp64_tflops": round(rate * 49 / 1e12, 3)}
        torch.cuda.empty_cache()
    return out


def graph_leg(pr, reps=5):
    """hipGraph replay of whole Parareal iterations (PR_FLAG_GRAPH) against eager
    launches: the 65^2 FP64 configuration (numerical G 33^2, N = 8; every kernel a
    few microseconds, so launch cost dominates) and a 129^2 FP32 one (N = 64,
    same-grid implicit G, seeds 0-3).  Median of `reps` solves each after a
    warm-up solve (which captures)."""
    import statistics
    import torch
    from synthetic import plain_at_scale, plain_fp64
    cases = {"fp64_65": [(plain_fp64(), pr.PR_G_NUMERICAL)],
             "fp32_129_lod": [(plain_at_scale(s, M=129, n_slices=64, coarse_M=33)
                               .replace(coarse_steps_per_slice=4), pr.PR_G_LOD) for s in range(4)]}
    res = {"workload": "eager launches vs one captured graph per Parareal iteration: "
                       "65^2 FP64 (numerical G 33^2, N=8) and 129^2 FP32 (LOD G, N=64, seeds 0-3)"}
    for case, items in cases.items():
        row = {}
        for name, flags in (("eager", 0), ("graph", pr.PR_FLAG_GRAPH)):
            ms, iters = [], []
            for inst, kind in items:
                sv = pr.Solver(inst, coarse_kind=kind, flags=flags)
                sv.solve()
                torch.cuda.synchronize()
                t = []
                for _ in range(reps):
                    a = time.perf_counter()
                    r = sv.solve()
                    t.append((time.perf_counter() - a) * 1e3)
                ms.append(statistics.median(t))
                iters.append(r.iters)
                sv.close()
            row[name] = {"median_ms": [round(x, 3) for x in ms], "iters": iters}
        row["speedup"] = round(sum(row["eager"]["median_ms"]) / sum(row["graph"]["median_ms"]), 3)
        res[case] = row
    return res


def step_probe(pr, M=2049, n_slices=32):
    """The step kernel alone at one shape: an M^2 grid with the parameters of the
    largest single solve and slices of its length (2/256, so 7207 explicit steps
    per slice at 2049^2 and 1802 at 1025^2), one Parareal iteration (the fine
    sweep over all slices; the same-grid implicit G), solved twice (warm-up,
    then measured).  Reports the HIP-event time of the step launches as point-
    steps/s, as 12 B per point-step (the unfused algorithmic bytes) and as the
    25 FP32 operations per point-step of the update."""
    import torch
    from synthetic import largest_single
    inst = largest_single().replace(M=M, n_slices=n_slices, T=2.0 * n_slices / 256,
                                    coarse_steps_per_slice=4)
    sv = pr.Solver(inst, coarse_kind=pr.PR_G_LOD, flags=pr.PR_FLAG_TIME_STEPS, max_iters=1)
    sv.solve()
    torch.cuda.synchronize()
    r = sv.solve()
    st = r.stats
    sv.close()
    pts = st["timed_step_bytes"] / 12.0 / (st["t_step_kernels_ms"] * 1e-3)
    return {"workload": "%d^2 FP32 increment form, %d slices of dT = 2/256, %d explicit steps "
                        "per slice, one fine sweep" % (M, n_slices, st["fine_steps"]),
            "point_steps_per_s": round(pts, 1),
            "effective_gbs": round(pts * 12.0 / 1e9, 1),
            "achieved_tflops": round(pts * FLOPS_PER_POINT_STEP / 1e12, 3),
            "step_launches": st["fine_step_launches"], "timed_launches": st["timed_step_launches"],
            "avg_launch_us": round(st["t_step_kernels_ms"] * 1e3 / max(1, st["timed_step_launches"]), 2),
            "point_steps_per_launch": round(st["timed_step_bytes"] / 12.0 / max(1, st["timed_step_launches"]))}


def largest_share_leg(pr):
    """One GPU's share of the largest solve: 2049^2, 32 of its 256 slices."""
    return step_probe(pr, 2049, 32)


def fno_flops_per_sample():
    """Algorithmic FLOPs of one forward pass of the operator (multiply-adds x 2):
    lift, four Fourier layers (pointwise W, truncated DFTs as real products,
    per-mode mixing, inverse DFTs) and projection."""
    P = 64 * 64
    lift = 2 * P * (7 * 64 + 64 * 32)
    layer = (2 * P * 32 * 32 + 2 * 64 * 24 * 64 * 32 + 2 * 24 * 24 * 128 * 32
             + 2 * 576 * 64 * 32 + 2 * 12 * 128 * 48 * 32 + 2 * 64 * 64 * 24 * 32)
    proj = 2 * P * (32 * 128 + 128)
    return lift + 4 * layer + proj


def fno_leg(pr, insts, seeds, serial_ref, train_s, parareal=True):
    """Neural coarse propagator: 20,032 pairs from serial F on 313 seed-drawn 257^2
    trajectories (N = 64, T = 1), BF16 training for a fixed budget, then Parareal
    with the trained operator as G on the bench instances (LOD fallback on)."""
    import torch
    from paper_2404_02521_amd import _lib as L
    from paper_2404_02521_amd.fno import Fno
    from paper_2404_02521_amd.train import evaluate, generate_pairs, init_params, train
    from synthetic import plain_at_scale
    dT = 1.0 / 64
    t = time.perf_counter()
    pairs, meta = generate_pairs([plain_at_scale(1000 + i, M=257) for i in range(313)])
    vp, vm = generate_pairs([plain_at_scale(2000 + i, M=257) for i in range(4)])
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t
    flat = init_params(0).cuda()
    net = Fno(max_batch=64, out_scale=dT)
    net.set_params(flat)
    zero = Fno(max_batch=64, out_scale=dT)
    zero.set_params(torch.zeros_like(flat))
    v_zero = evaluate(zero, vp, vm, dT)
    v_init = evaluate(net, vp, vm, dT)
    zero.close()
    hist = train(net, pairs, meta, dT, 10 ** 6, 64, L.PR_FNO_BF16, log_every=1000,
                 time_budget_s=train_s)
    steps, t_train = hist[-1][1], hist[-1][-1]
    v_tr = evaluate(net, vp, vm, dT)
    flops = 3.0 * fno_flops_per_sample() * 64 * steps
    params = net.params()
    net.close()
    # the learned G alone (no fallback), six iterations per instance: its own
    # increments, whether it converges and its error against serial F
    own = {"iters": [], "status": [], "increments": [], "err": []}
    for s_, inst in zip(seeds, insts) if parareal else []:
        fi = Fno(max_batch=1, out_scale=dT)
        fi.set_params(params)
        sv = pr.Solver(inst, coarse_kind=pr.PR_G_FNO, max_iters=6, flags=pr.PR_FLAG_NO_FALLBACK)
        sv.attach_fno(fi)
        try:
            r = sv.solve()
            own["iters"].append(r.iters)
            own["status"].append(r.status)
            own["increments"].append([float("%.3g" % x) for x in r.increments])
            ref = serial_ref[s_]
            own["err"].append(float("%.3g" % float((r.value - ref).abs().max() / ref.abs().max())))
        except pr.PararealError as e:   # a non-finite increment ends the solve
            own["iters"].append(None)
            own["status"].append(e.status)
            own["increments"].append(None)
            own["err"].append(None)
        sv.close()
        fi.close()
    res = {"K": [], "ms": [], "err": [], "fallback": []}
    for s_, inst in zip(seeds, insts) if parareal else []:
        fi = Fno(max_batch=1, out_scale=dT)
        fi.set_params(params)
        sv = pr.Solver(inst, coarse_kind=pr.PR_G_FNO)
        sv.attach_fno(fi)
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = sv.solve()
        res["ms"].append(round((time.perf_counter() - a) * 1e3, 1))
        res["K"].append(r.iters)
        res["fallback"].append(r.stats["coarse_fallback"])
        ref = serial_ref[s_]
        res["err"].append(float((r.value - ref).abs().max() / ref.abs().max()))
        sv.close()
        fi.close()
    return {"workload": "FNO width 32, 4 layers, 12x12 modes, 64^2, BF16 MFMA training on %d pairs "
                        "(313 seed-drawn 257^2 F trajectories, N=64) for %.0f s; then G on the "
                        "513^2 bench instances through DST transfers" % (pairs.shape[0], train_s),
            "data_s": round(t_data, 2), "train_steps": steps, "train_s": round(t_train, 2),
            "train_samples_per_s": round(64 * steps / t_train, 1),
            "train_tflops": round(flops / t_train / 1e12, 3),
            "train_mfma_frac_bf16": round(flops / t_train / 2.5e15, 5),
            "val_data_mse": {"untrained": v_init[1], "without_network": v_zero[1],
                             "trained": v_tr[1]},
            "parareal_fno_g_only": None if not parareal else dict(
                own, note="PR_FLAG_NO_FALLBACK, max_iters 6: the learned G's own iteration "
                          "(status 5 = stopped at max_iters above tolerance)",
                finished_on_fno_g=sum(1 for st_ in own["status"] if st_ == 0)),
            "parareal_with_fallback": None if not parareal else {
                "iters": res["K"], "ms": res["ms"], "max_err_vs_serial_f": max(res["err"]),
                "coarse_fallback": res["fallback"],
                "note": "a solve that fell back (coarse_fallback 1) finished on the LOD G; its "
                        "time includes the abandoned FNO-G iterations",
                "solves_per_s_including_fallbacks": round(len(res["ms"]) / (sum(res["ms"]) * 1e-3), 4)}}


def serving_leg(pr, count=120, seed=11, sides=(129, 257)):
    """Independent solves (seed-drawn parameters, T ~ U[0.25, 2], N in {16, 32, 64},
    grid side uniform over `sides`) through the continuous-batching server with
    the same-grid implicit coarse propagator: first all requests at once (the
    saturation throughput S), then Poisson arrivals at 0.5 S and 0.9 S with the
    same request draws, reporting p50 / p99 latency (submit to result)."""
    import torch
    from paper_2404_02521_amd.serve import Server, run_poisson
    from synthetic import serving_requests
    _, insts = serving_requests(1.0, count, seed=seed, sides=sides)
    out = {"workload": "%d requests, sides %s, N in {16,32,64}, T~U[0.25,2], LOD coarse "
                       "propagator; saturation, then Poisson at 0.5x and 0.9x of it"
                       % (count, list(sides))}
    sv = Server(64 << 30, max_resident=64, n_streams=8)
    r = run_poisson(sv, [0.0] * count, insts)
    sat = r["solves_per_s"]
    out["saturation"] = {"solves_per_s": round(sat, 2), "p50_ms": round(r["p50_ms"], 2),
                         "p99_ms": round(r["p99_ms"], 2), "peak_resident": r["peak_resident"]}
    for frac in (0.5, 0.9):
        t, _ = serving_requests(frac * sat, count, seed=seed, sides=sides)
        r = run_poisson(sv, t, insts)
        out["poisson_%.1fx" % frac] = {"rate": round(frac * sat, 2),
                                       "solves_per_s": round(r["solves_per_s"], 2),
                                       "p50_ms": round(r["p50_ms"], 2),
                                       "p99_ms": round(r["p99_ms"], 2),
                                       "mean_iters": round(sum(r["iters"]) / count, 2),
                                       "peak_resident": r["peak_resident"]}
    # the same requests with the fine sweeps of each scheduling pass in shared
    # (ragged) launches: saturation and the same Poisson arrivals
    sr = Server(64 << 30, max_resident=64, n_streams=8, ragged=True)
    r = run_poisson(sr, [0.0] * count, insts)
    rg = {"saturation": {"solves_per_s": round(r["solves_per_s"], 2),
                         "p50_ms": round(r["p50_ms"], 2), "p99_ms": round(r["p99_ms"], 2)}}
    for frac in (0.5, 0.9):
        t, _ = serving_requests(frac * sat, count, seed=seed, sides=sides)
        r = run_poisson(sr, t, insts)
        rg["poisson_%.1fx" % frac] = {"rate": round(frac * sat, 2),
                                      "solves_per_s": round(r["solves_per_s"], 2),
                                      "p50_ms": round(r["p50_ms"], 2),
                                      "p99_ms": round(r["p99_ms"], 2)}
    st = sr.ragged_stats()
    rg["shared_launches"] = st["launches"]
    rg["requests_per_launch"] = round(st["entries"] / max(1, st["launches"]), 2)
    rg["note"] = ("PR_SERVER_RAGGED_F: the fine sweeps of the requests ready in one scheduling "
                  "pass share step launches (up to 8 requests each, sweeps bucketed by work "
                  "per step, a stream per bucket)")
    out["ragged_fine_launches"] = rg
    sr.close()
    # the full grid-size mix at saturation only: 1025^2 requests take seconds each
    _, full = serving_requests(1.0, 32, seed=seed + 1, sides=(129, 257, 513, 1025))
    r = run_poisson(sv, [0.0] * len(full), full)
    out["full_mix_saturation"] = {"sides": [129, 257, 513, 1025], "count": len(full),
                                  "solves_per_s": round(r["solves_per_s"], 3),
                                  "p50_ms": round(r["p50_ms"], 1), "p99_ms": round(r["p99_ms"], 1),
                                  "peak_resident": r["peak_resident"],
                                  "peak_arena_gb": round(r["peak_arena_bytes"] / 2 ** 30, 2)}
    sv.close()
    # offered loads of 50 to 2000 requests/s, one second of Poisson arrivals each,
    # with load shedding (PR_EBUSY beyond the queue bound): on the full mix (16
    # resident, 16 waiting) and on the {129, 257} sub-mix (64 and 64), where the
    # rates lie on both sides of saturation
    for key, sides_r, cap in (("offered_load_full_mix", (129, 257, 513, 1025), 16),
                              ("offered_load_129_257", sides, 64)):
        rates = {}
        for rate in (50.0, 100.0, 200.0, 500.0, 1000.0, 2000.0):
            t, insts_r = serving_requests(rate, int(rate), seed=seed + 2, sides=sides_r)
            sq = Server(64 << 30, max_resident=cap, n_streams=8, max_queued=cap)
            r = run_poisson(sq, t, insts_r)
            row = {"offered_per_s": rate, "arrivals": int(rate), "served": r["served"],
                   "rejected": r["rejected"], "solves_per_s": round(r["solves_per_s"], 3)}
            if r["served"]:
                row.update(p50_ms=round(r["p50_ms"], 1), p99_ms=round(r["p99_ms"], 1),
                           peak_resident=r["peak_resident"])
            rates["%g_per_s" % rate] = row
            sq.close()
            progress("serving %s at %g req/s done" % (key, rate))
        out[key] = dict(rates, note="one second of Poisson arrivals per rate; queue bound %d "
                                    "(refused beyond), %d resident; latency of the served "
                                    "requests, arrival to result; solves/s over the served "
                                    "requests' span" % (cap, cap))
    torch.cuda.empty_cache()
    return out


def run_cpu_baseline(insts, K_gpu):
    """The FP64 oracle on the host cores, on a bounded sample of the workload.

    Measured: the oracle's complete serial F of the seed-3 instance (the
    cheapest of the eight: 64 slices x 283 explicit steps on 513^2) with every
    host thread on the rows; the workload's solves/s follows by scaling that
    point-step rate to the mean serial-F point-steps of the eight instances (the
    exact answer the GPU's Parareal solves approximate to 1e-5).  Also reported:
    the oracle's own Parareal on seed 0 (initial sweep + one iteration
    measured, a K-iteration solve extrapolated as init + K * iter)."""
    import oracle
    from paper_2404_02521_amd.parareal import plan

    def prob(inst, M=None):
        return oracle.Problem(M=M or inst.M, sigma1=inst.sigma1, sigma2=inst.sigma2,
                              rho=inst.rho, r=inst.r, payoff_kind=inst.payoff, w1=inst.w1,
                              w2=inst.w2, strike=inst.strike)

    sample = insts[3] if len(insts) > 3 else insts[0]
    mf_s = plan(sample)[0]
    t = time.perf_counter()
    oracle.serial_fine(prob(sample), sample.n_slices, sample.T, mf_s)
    t_ser = time.perf_counter() - t
    pts = sample.n_slices * mf_s * (sample.M - 2) ** 2
    rate = pts / t_ser
    mean_pts = sum(i.n_slices * plan(i)[0] * (i.M - 2) ** 2 for i in insts) / len(insts)
    inst = insts[0]
    mf, mg, _, _ = plan(inst)
    pf, pc = prob(inst), prob(inst, inst.coarse_M)
    t = time.perf_counter()
    oracle.parareal_bs(pf, pc, inst.n_slices, inst.T, mf, mg, max_iters=0, tol=0.0)
    t_init = time.perf_counter() - t
    t = time.perf_counter()
    oracle.parareal_bs(pf, pc, inst.n_slices, inst.T, mf, mg, max_iters=1, tol=0.0)
    t_one = time.perf_counter() - t
    t_iter = max(t_one - t_init, 1e-9)
    return {"value": round(rate / mean_pts, 6), "unit": "solves/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "FP64 oracle serial F, complete solve of the seed-3 513^2 instance "
                      "(64 slices x %d steps, %.3g point-steps) in %.2f s measured on %d host "
                      "threads (rows in parallel), %.3g point-steps/s; scaled to the mean "
                      "serial-F work of seeds 0-7 (%.3g point-steps); host %s"
                      % (mf_s, pts, t_ser, oracle.num_threads(), rate, mean_pts,
                         host_cpu_model()),
            "measured_s": round(t_ser, 3), "point_steps_per_s": round(rate, 1),
            "parareal_extrapolated": {
                "solves_per_s": round(1.0 / (t_init + K_gpu * t_iter), 6),
                "how": "oracle Parareal on seed 0 (OpenMP over slices): init %.2f s + one "
                       "iteration %.2f s measured, a solve taken as init + K*iter with the "
                       "GPU's K=%d (not measured end to end)" % (t_init, t_iter, K_gpu)}}


if __name__ == "__main__":
    main()
