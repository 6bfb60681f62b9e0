"""parareal_solve_static (the entry point that allocates nothing) against
parareal_create + parareal_solve on the same problems, through the C ABI.

Both run the same kernels with the same launch geometry, so the results must
be equal bitwise; two calls in a row, the second on a smaller problem, check
that what the first call left in the shared static scratch does not leak into
the second.
"""
import gc

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2404_02521_amd as pr_
    return pr_


def _pair(pr, inst, **kw):
    import torch
    from paper_2404_02521_amd.parareal import solve_static
    ref = pr.Solver(inst, **kw)
    want = ref.solve()
    out = torch.empty((inst.M, inst.M), dtype=torch.float64, device="cuda")
    gc.collect()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    got = solve_static(inst, out=out, **kw)
    torch.cuda.synchronize()
    # nothing new on torch's allocator (earlier tests' garbage may be freed meanwhile)
    assert torch.cuda.memory_allocated() <= before
    assert got.status == want.status
    assert got.iters == want.iters
    assert got.increments == want.increments
    assert np.array_equal(got.value.cpu().numpy(), want.value.cpu().numpy())
    ref.close()
    return got


def test_static_matches_create_solve_twice(pr):
    from helpers import say
    from synthetic import plain_at_scale, plain_fp64
    big = plain_at_scale(2, M=257, n_slices=16, coarse_M=65).replace(T=0.25)
    small = plain_fp64()
    say("static scratch: 257^2 x 16 FP32, then 65^2 x 8 FP64")
    g1 = _pair(pr, big)
    g2 = _pair(pr, small)
    assert g1.stats["workspace_bytes"] > g2.stats["workspace_bytes"]
    # the LOD coarse propagator through the same entry point
    say("static scratch: 129^2 x 16 FP32 LOD")
    _pair(pr, plain_at_scale(1, M=129, n_slices=16, coarse_M=33).replace(T=0.5),
          coarse_kind=pr.PR_G_LOD)


def test_static_rejects_oversize(pr):
    from paper_2404_02521_amd.parareal import solve_static
    from synthetic import plain_at_scale
    inst = plain_at_scale(0)   # 513^2 x 64 slices: about 0.3 GB of workspace
    with pytest.raises(pr.PararealError) as e:
        solve_static(inst)
    assert e.value.status == pr._lib.PR_ENOMEM
