"""Continuous-batching server: each result is the same alone and in the mix
(bitwise: per-request kernels are deterministic and independent), admission
respects the arena, failures are reported per request."""
import numpy as np
import pytest

from helpers import say
from synthetic import plain_at_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pr():
    import torch
    assert torch.cuda.is_available()
    import paper_2404_02521_amd as pr_
    return pr_


def host(t):
    return t.detach().cpu().numpy()


def mix():
    out = []
    for k, (M, N, Mc) in enumerate([(65, 8, 33), (129, 16, 33), (65, 16, 17), (129, 8, 65),
                                    (97, 8, 33), (129, 16, 33)]):
        inst = plain_at_scale(100 + k, M=M, n_slices=N, coarse_M=Mc).replace(T=0.25 + 0.1 * k)
        out.append((inst, "lod" if k % 2 == 0 else "num"))
    return out


def test_alone_vs_mix(pr):
    from paper_2404_02521_amd.serve import Server
    reqs = mix()
    kinds = {"lod": pr.PR_G_LOD, "num": pr.PR_G_NUMERICAL}
    say("serving mix", len(reqs))
    sv = Server(2 << 30, max_resident=4, n_streams=3)
    ids = [sv.submit(inst, kinds[k]) for inst, k in reqs]
    infos = sv.drain(ids, timeout_s=300)
    for rid, (inst, k) in zip(ids, reqs):
        alone = pr.Solver(inst, coarse_kind=kinds[k]).solve()
        assert infos[rid]["status"] in (0, 5)
        assert infos[rid]["iters"] == alone.iters
        assert np.array_equal(host(sv.result(rid)), host(alone.value)), (inst.M, k)
    assert sv.peaks()[0] <= 4
    sv.close()


def test_admission_by_footprint(pr):
    from paper_2404_02521_amd.serve import Server
    reqs = [plain_at_scale(200 + k, M=129, n_slices=16, coarse_M=33) for k in range(5)]
    fp = Server.footprint(reqs[0])
    say("admission", fp)
    sv = Server(2 * fp + 1024, max_resident=8, n_streams=4)
    ids = [sv.submit(inst) for inst in reqs]
    infos = sv.drain(ids, timeout_s=300)
    peak, peak_bytes = sv.peaks()
    assert peak <= 2 and peak_bytes <= 2 * fp + 1024
    assert all(i["status"] == 0 for i in infos.values())
    # later requests waited in the queue for memory
    assert max(i["queue_ms"] for i in infos.values()) > 0.0
    for rid, inst in zip(ids, reqs):
        alone = pr.Solver(inst, coarse_kind=pr.PR_G_LOD).solve()
        assert np.array_equal(host(sv.result(rid)), host(alone.value))
    sv.close()


def test_rejects_and_statuses(pr):
    from paper_2404_02521_amd.serve import Server
    small = plain_at_scale(300, M=65, n_slices=8, coarse_M=33)
    big = plain_at_scale(301, M=257, n_slices=16, coarse_M=65)
    say("rejects")
    sv = Server(Server.footprint(small) + 4096, max_resident=2, n_streams=1)
    with pytest.raises(pr.PararealError) as e:
        sv.submit(big)
    assert e.value.status == 3   # PR_ENOMEM
    with pytest.raises(pr.PararealError) as e:
        sv.submit(small.replace(rho=1.5))
    assert e.value.status == 1   # PR_EINVAL
    rid = sv.submit(small, max_iters=1)
    info = sv.drain([rid])[rid]
    assert info["status"] == 5 and info["iters"] == 1   # PR_ENOTCONV, result still written
    alone = pr.Solver(small, coarse_kind=pr.PR_G_LOD, max_iters=1).solve()
    assert np.array_equal(host(sv.result(rid)), host(alone.value))
    sv.close()
