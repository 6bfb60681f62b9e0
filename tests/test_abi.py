"""C-ABI checks that need no GPU: symbols, struct layouts, planning, validation."""
import ctypes as C
import os
import re
import subprocess

import pytest

import oracle
from paper_2404_02521_amd import _lib as L
from paper_2404_02521_amd.parareal import make_structs, plan
from synthetic import plain_fp64, plain_at_scale, largest_single, BASKET, EXCHANGE

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "parareal.h")


def declared_functions():
    """Every entry point declared in include/*.h."""
    names = set()
    for h in (HEADER, os.path.join(ROOT, "include", "parareal3.h")):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b((?:parareal|pr_server|pr_fno|pr3)_\w+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert {n for n, _, _ in L.SIGNATURES} == set(names)
    assert lib.parareal_abi_version() == 2


def test_constants_match_header(tmp_path):
    """Every PR_* constant of the header (#define or enum) that the binding
    mirrors has the value the C compiler gives it; the option flags, kinds and
    status codes are all mirrored."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    names = set(re.findall(r"#define\s+(PR_[A-Z0-9_]+)\s", src))
    names |= set(re.findall(r"\b(PR_[A-Z0-9_]+)\s*=", src))
    names.discard("PR_H")
    must = {n for n in names if re.match(r"PR_(FLAG|SERVER|PAYOFF|BC|G|FINE|FP|OP|E|OK|FNO_BASE)", n)}
    assert {"PR_FLAG_SERIAL_CHAIN", "PR_G_IMPLICIT", "PR_PAYOFF_CASH_OR_NOTHING"} <= must
    for n in must:
        assert hasattr(L, n), n
    mirrored = sorted(n for n in names if hasattr(L, n))
    body = "".join('printf("%%s %%lld\\n", "%s", (long long)(%s));' % (n, n) for n in mirrored)
    c = tmp_path / "k.c"
    c.write_text('#include <stdio.h>\n#include "%s"\nint main(void){%s return 0;}\n' % (HEADER, body))
    exe = tmp_path / "k"
    subprocess.run(["gcc", "-o", str(exe), str(c)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = dict(line.split() for line in out.strip().splitlines())
    for n in mirrored:
        assert int(got[n]) == int(getattr(L, n)), n


def test_struct_layouts_match_header(tmp_path):
    """sizeof / offsetof from the C compiler against the ctypes mirrors."""
    structs = {"pr_grid": L.pr_grid, "pr_model": L.pr_model, "pr_payoff": L.pr_payoff,
               "pr_options": L.pr_options, "pr_stats": L.pr_stats,
               "pr_server_options": L.pr_server_options, "pr_request_info": L.pr_request_info,
               "pr_fno_config": L.pr_fno_config, "pr_fno_file_info": L.pr_fno_file_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', 'int main(void){']
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} %zu\\n", sizeof({sname}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{sname}.{f} %zu\\n", offsetof({sname}, {f}));')
    lines.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-o", str(exe), str(c)])
    out = dict(l.rsplit(" ", 1) for l in subprocess.check_output([str(exe)]).decode().split("\n") if l)
    for sname, cls in structs.items():
        assert int(out[sname]) == C.sizeof(cls), sname
        for f, _ in cls._fields_:
            assert int(out[f"{sname}.{f}"]) == getattr(cls, f).offset, (sname, f)


def _oracle_problem(inst, M=None):
    return oracle.Problem(M=M or inst.M, sigma1=inst.sigma1, sigma2=inst.sigma2, rho=inst.rho,
                          r=inst.r, payoff_kind=inst.payoff, w1=inst.w1, w2=inst.w2,
                          strike=inst.strike, s_max=inst.s_max)


@pytest.mark.parametrize("seed", range(6))
def test_plan_agrees_with_oracle(seed):
    """Library and oracle derive the step counts independently (Gershgorin at 0.9)."""
    inst = plain_at_scale(seed)
    mf, mg, dsf, dsc = plan(inst)
    dT = inst.T / inst.n_slices
    assert mf == oracle.steps_for(_oracle_problem(inst), dT, inst.cfl)
    assert mg == oracle.steps_for(_oracle_problem(inst, inst.coarse_M), dT, inst.cfl)
    assert abs(dsf - oracle.stable_dt(_oracle_problem(inst))) <= 1e-15 * dsf
    assert 91 <= mf <= 2800


def test_plan_fixed_counts_c1():
    inst = plain_fp64()
    mf, mg, _, _ = plan(inst)
    assert (mf, mg) == (128, 64)
    big = largest_single()                          # 2049^2 fine, 257^2 coarse
    mf, mg, _, _ = plan(big)
    assert mf == 7207 and mg > 100


def _create(inst, nbytes=1 << 20, ptr=256, **kw):
    g, m, p, o = make_structs(inst, **kw)
    h = C.c_void_p()
    return L.lib().parareal_create(C.byref(g), C.byref(m), C.byref(p), C.byref(o),
                                   C.c_void_p(ptr), C.c_uint64(nbytes), None, C.byref(h))


def test_validation_before_any_gpu_call():
    inst = plain_fp64()
    assert _create(inst.replace(M=3)) == L.PR_EINVAL
    assert _create(inst.replace(n_slices=0)) == L.PR_EINVAL
    assert _create(inst.replace(sigma1=-0.1)) == L.PR_EINVAL
    assert _create(inst.replace(rho=1.0)) == L.PR_EINVAL
    assert _create(inst.replace(T=0.0)) == L.PR_EINVAL
    assert _create(inst.replace(coarse_M=30)) == L.PR_EINVAL          # 64 % 29 != 0
    assert _create(inst.replace(M=1025, coarse_M=513)) == L.PR_EINVAL   # coarse above 257
    g1, _, _, o1 = make_structs(inst.replace(M=1025, coarse_M=257))
    assert L.lib().parareal_workspace_bytes(C.byref(g1), C.byref(o1)) > 0
    assert _create(inst.replace(fine_steps_per_slice=8)) == L.PR_EUNSTABLE
    assert _create(inst.replace(coarse_steps_per_slice=2)) == L.PR_EUNSTABLE
    assert _create(inst, nbytes=16) == L.PR_ENOMEM
    assert _create(inst, ptr=0) == L.PR_ENOMEM
    assert _create(inst.replace(strike=float("nan"))) == L.PR_EINVAL
    assert _create(inst, bc_kind=L.PR_BC_EXACT) == L.PR_EINVAL         # basket with w2 != 0
    g, m, p, o = make_structs(inst)
    assert L.lib().parareal_workspace_bytes(C.byref(g), C.byref(o)) > 0
    g2, _, _, o2 = make_structs(inst.replace(M=4))
    assert L.lib().parareal_workspace_bytes(C.byref(g2), C.byref(o2)) == 0
    assert L.lib().parareal_strerror(L.PR_ENOMEM) == b"workspace too small"


def test_workspace_size_formula():
    """Workspace at the at-scale shape: two FP64 state stacks plus three FP32 increment
    stacks, with 512-element padded rows; fits easily in 288 GB even at 2049^2 x 256."""
    inst = plain_at_scale(0)
    g, _, _, o = make_structs(inst)
    nbytes = L.lib().parareal_workspace_bytes(C.byref(g), C.byref(o))
    per = 511 * 512
    assert nbytes >= 2 * 65 * per * 8 + 3 * 64 * per * 4
    # coarse per-slice arrays: Gold, d_n and the gathered F at coincident nodes (FP64)
    assert nbytes < 1.01 * (2 * 65 * per * 8 + 3 * 64 * per * 4) + 64 * 129 * 129 * 24 + 4096
    big = largest_single()
    g, _, _, o = make_structs(big)
    assert L.lib().parareal_workspace_bytes(C.byref(g), C.byref(o)) < 40e9


def test_fno_host_side_validation():
    """pr_fno_* argument checks that run before any GPU call."""
    lib = L.lib()
    assert lib.pr_fno_param_count() == 2370465
    assert lib.pr_fno_workspace_bytes(0) == 0
    assert lib.pr_fno_workspace_bytes(L.PR_FNO_MAX_BATCH + 1) == 0
    small, big = lib.pr_fno_workspace_bytes(1), lib.pr_fno_workspace_bytes(64)
    assert 0 < small < big
    h = C.c_void_p()
    bad = [L.pr_fno_config(0, L.PR_FNO_FP32, 1.0, L.PR_FNO_BASE_IDENTITY, 0),
           L.pr_fno_config(1, 7, 1.0, L.PR_FNO_BASE_IDENTITY, 0),
           L.pr_fno_config(1, L.PR_FNO_FP32, 0.0, L.PR_FNO_BASE_IDENTITY, 0),
           L.pr_fno_config(1, L.PR_FNO_FP32, 1.0, 9, 0)]
    for cfg in bad:
        assert lib.pr_fno_create(C.byref(cfg), None, 0, None, C.byref(h)) == L.PR_EINVAL
    ok = L.pr_fno_config(1, L.PR_FNO_FP32, 1.0, L.PR_FNO_BASE_FINE_LOD, 0)
    assert lib.pr_fno_create(C.byref(ok), None, 0, None, C.byref(h)) == L.PR_ENOMEM
    assert lib.pr_fno_create(C.byref(ok), C.c_void_p(256), small - 1, None,
                             C.byref(h)) == L.PR_ENOMEM
    assert lib.pr_fno_forward(None, None, None, 1, 0, None) == L.PR_EINVAL
    assert lib.pr_fno_destroy(None) == L.PR_EINVAL


def test_fno_coarse_kind_validation():
    """PR_G_FNO needs n >= 64 (the server's refusal without an attached operator
    is a GPU test: a server owns streams)."""
    inst = plain_at_scale(0, M=33, n_slices=8, coarse_M=9)
    g, m, p, o = make_structs(inst, L.PR_G_FNO)
    assert L.lib().parareal_workspace_bytes(C.byref(g), C.byref(o)) == 0
    inst = plain_at_scale(0, M=129, n_slices=8, coarse_M=33)
    g, m, p, o = make_structs(inst, L.PR_G_FNO)
    assert L.lib().parareal_workspace_bytes(C.byref(g), C.byref(o)) > 0
    rid = C.c_int64()
    assert L.lib().pr_server_submit(None, C.byref(g), C.byref(m), C.byref(p), C.byref(o),
                                    C.c_void_p(1), C.byref(rid)) == L.PR_EINVAL
    assert L.lib().pr_server_attach_fno(None, None) == L.PR_EINVAL
