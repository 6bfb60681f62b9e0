"""Bench-size results against the FP64 oracle's stored serial fine solutions.

tests/golden/make_bench_oracle.py wrote them from oracle/ alone: serial F of
the 513^2 x 64-slice at-scale problems (seeds 0-7, every 4th node) and of the
2049^2 x 256-slice single solve (every 8th node).  The CPU tests re-run the
cheapest seed through the oracle and check the record; the GPU tests hold the
GPU's serial F and Parareal results at these sizes to 1e-5 relative max-norm
of the oracle (FP32 increments over 18k-110k explicit steps).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from helpers import oproblem, rel_max, say
from synthetic import largest_single, plain_at_scale

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
META = json.load(open(os.path.join(HERE, "bench_oracle.json")))
FP32_TOL = 1e-5


def golden(name):
    return np.load(os.path.join(HERE, name))


def test_records_match_their_metadata():
    for name, m in META.items():
        a = golden(name)
        assert list(a.shape) == m["shape"], name
        assert hashlib.sha256(a.tobytes()).hexdigest() == m["sha256"], name
        inst = largest_single() if name.startswith("c5") else plain_at_scale(int(name[-5]))
        for k in ("M", "n_slices", "T", "sigma1", "sigma2", "rho", "r", "w1", "w2", "strike"):
            assert m[k] == getattr(inst, k), (name, k)


def test_c2_seed3_reproduced_by_the_oracle():
    """The cheapest seed (283 steps per slice) recomputed: bitwise the stored record."""
    inst = plain_at_scale(3)
    m = META["c2_serial_f_seed3.npy"]
    u = oracle.serial_fine(oproblem(inst), inst.n_slices, inst.T, m["fine_steps_per_slice"])
    assert np.array_equal(u[::4, ::4], golden("c2_serial_f_seed3.npy"))


@pytest.mark.gpu
@pytest.mark.parametrize("seed", [0, 3])
def test_bench_size_against_oracle(seed):
    """513^2 x 64 slices, the bench's configuration: serial F and the Parareal
    result (numerical G on 129^2, relative stop 1e-7) within 1e-5 of the oracle."""
    import paper_2404_02521_amd as pr
    inst = plain_at_scale(seed)
    say("bench size vs oracle", seed)
    s = pr.Solver(inst)
    ser = s.serial_fine().value.cpu().numpy()[::4, ::4]
    par = s.solve().value.cpu().numpy()[::4, ::4]
    ref = golden("c2_serial_f_seed%d.npy" % seed)
    assert rel_max(ser, ref) <= FP32_TOL
    assert rel_max(par, ref) <= FP32_TOL
    s.close()
