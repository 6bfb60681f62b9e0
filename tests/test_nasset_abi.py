"""Three-asset boundary checks that need no GPU: step planning against the
oracle's Gershgorin bound, validation, and the struct layouts."""
import ctypes as C
import os
import subprocess

import pytest

from oracle import nasset as na
from paper_2404_02521_amd import _lib as L
from paper_2404_02521_amd.nasset import make_problem, plan
from synthetic import three_asset

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def oproblem(inst, M=None):
    return na.Problem3(M=M or inst.M, sigma=inst.sigma, rho=inst.rho, r=inst.r, w=inst.w,
                       strike=inst.strike, s_max=inst.s_max)


@pytest.mark.parametrize("seed,M,Mc,N", [(0, 65, 17, 16), (1, 33, 9, 4), (2, 129, 33, 8),
                                          (3, 17, 5, 2)])
def test_plan_matches_the_oracle_bound(seed, M, Mc, N):
    inst = three_asset(seed, M=M, coarse_M=Mc, n_slices=N)
    mf, mg = plan(inst)
    dT = inst.T / N
    assert mf == na.steps_for(oproblem(inst), dT, 0.9)
    assert mg == na.steps_for(oproblem(inst, Mc), dT, 0.9)


def test_validation():
    good = three_asset(0, M=17, coarse_M=5, n_slices=2)
    assert L.lib().pr3_workspace_bytes(C.byref(make_problem(good))) > 0
    bad = [good.replace(coarse_M=6),                 # (n - 1) not divisible
           good.replace(rho=(0.9, 0.9, -0.9)),       # not positive semi-definite
           good.replace(sigma=(0.2, 0.0, 0.3)),
           good.replace(n_slices=0), good.replace(M=3)]
    for b in bad:
        p = make_problem(b)
        assert L.lib().pr3_plan(C.byref(p), None, None) == L.PR_EINVAL, b
        assert L.lib().pr3_workspace_bytes(C.byref(p)) == 0
    unstable = good.replace(fine_steps=1)
    assert L.lib().pr3_plan(C.byref(make_problem(unstable)), None, None) == L.PR_EUNSTABLE


def test_struct_layouts(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>',
             '#include "%s"' % os.path.join(ROOT, "include", "parareal3.h"), 'int main(void){']
    for name, cls in (("pr3_problem", L.pr3_problem), ("pr3_stats", L.pr3_stats)):
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, f, name, f))
    lines.append("return 0;}")
    src = tmp_path / "l.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "l"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for name, cls in (("pr3_problem", L.pr3_problem), ("pr3_stats", L.pr3_stats)):
        assert int(got[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got["%s.%s" % (name, f)]) == getattr(cls, f).offset, (name, f)
