"""HIP-graph replay of Parareal iterations against eager execution (bitwise).

Each graph is replayed several times, with eager work and synchronisations of
the program's own between the replays; every replay must equal the eager
result exactly."""
import numpy as np
import pytest

from helpers import say
from synthetic import BASKET, EXCHANGE, plain_at_scale, plain_fp64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pr():
    import torch
    assert torch.cuda.is_available()
    import paper_2404_02521_amd as pr_
    return pr_


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("case", ["c1_basket", "c1_exchange", "fp32_129", "g_equal_f"])
def test_graph_replay_matches_eager(pr, case):
    import torch
    kw = {}
    if case == "c1_basket":
        inst = plain_fp64(BASKET)
    elif case == "c1_exchange":
        inst = plain_fp64(EXCHANGE).replace(tol=0.0)
    elif case == "fp32_129":
        inst = plain_at_scale(5, M=129, n_slices=16, coarse_M=33)
        kw = dict(max_iters=4)
    else:
        inst = plain_fp64(EXCHANGE).replace(fp32=True)
        kw = dict(coarse_kind=pr.PR_G_FINE)
    say("graph replay", case)
    eager = pr.Solver(inst, **kw)
    ref = eager.solve()
    ref_v = host(ref.value)
    graph = pr.Solver(inst, flags=pr.PR_FLAG_GRAPH, **kw)
    for rep in range(3):
        res = graph.solve()
        assert res.iters == ref.iters
        assert np.array_equal(host(res.value), ref_v), rep
        assert res.increments == ref.increments
        # eager work of the program between replays
        other = eager.solve()
        torch.cuda.synchronize()
        assert np.array_equal(host(other.value), ref_v)
