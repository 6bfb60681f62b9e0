"""Continuous-batching server: each result is the same alone and in the mix
(bitwise: per-request kernels are deterministic and independent), also when
the requests' fine sweeps share ragged launches; served results match the FP64
oracle's serial F, admission respects the arena and the bounded queue,
failures are reported per request."""
import numpy as np
import pytest

import oracle
from helpers import oproblem, rel_max, say
from synthetic import BASKET, EXCHANGE, plain_at_scale, plain_fp64, serving_requests

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


@pytest.mark.parametrize("ragged", [False, True])
def test_alone_vs_mix(pr, ragged):
    from paper_2404_02521_amd.serve import Server
    reqs = mix()
    kinds = {"lod": pr.PR_G_LOD, "num": pr.PR_G_NUMERICAL}
    say("serving mix", len(reqs), "ragged" if ragged else "")
    sv = Server(2 << 30, max_resident=4, n_streams=3, ragged=ragged)
    ids = [sv.submit(inst, kinds[k]) for inst, k in reqs]
    infos = sv.drain(ids, timeout_s=300)
    for rid, (inst, k) in zip(ids, reqs):
        alone = pr.Solver(inst, coarse_kind=kinds[k]).solve()
        assert infos[rid]["status"] in (0, 5)
        assert infos[rid]["iters"] == alone.iters
        assert np.array_equal(host(sv.result(rid)), host(alone.value)), (inst.M, k)
    assert sv.peaks()[0] <= 4
    st = sv.ragged_stats()
    if ragged:
        assert st["launches"] >= 1 and st["entries"] >= st["launches"]
    else:
        assert st == {"ticks": 0, "launches": 0, "entries": 0}
    sv.close()


def test_ragged_fine_launches(pr):
    """PR_SERVER_RAGGED_F with every request admitted in the first pass: nine
    FP32 sweeps of five fused steps (more than one launch's eight entries), an
    FP64 request and an exact-ring request (its own launches) share the ticks;
    every result equals its solve alone bitwise, and the shared launches carried
    more than one request each on average."""
    from paper_2404_02521_amd.serve import Server
    B = pr.PR_BC_FORWARD_INTRINSIC
    reqs = [(inst, pr.PR_G_LOD if k == "lod" else pr.PR_G_NUMERICAL, B) for inst, k in mix()]
    reqs += [(plain_at_scale(510 + k, M=129, n_slices=32, coarse_M=33).replace(T=0.3),
              pr.PR_G_LOD, B) for k in range(3)]
    reqs.append((plain_fp64(BASKET), pr.PR_G_LOD, B))
    reqs.append((plain_fp64(EXCHANGE), pr.PR_G_NUMERICAL, pr.PR_BC_EXACT))
    say("ragged launches", len(reqs))
    sv = Server(4 << 30, max_resident=len(reqs), n_streams=3, ragged=True)
    ids = [sv.submit(inst, kind, bc_kind=bc) for inst, kind, bc in reqs]
    infos = sv.drain(ids, timeout_s=300)
    st = sv.ragged_stats()
    print("ragged stats", st)
    assert st["launches"] >= 1 and st["entries"] > st["launches"]
    for rid, (inst, kind, bc) in zip(ids, reqs):
        alone = pr.Solver(inst, coarse_kind=kind, bc_kind=bc).solve()
        assert infos[rid]["status"] in (0, 5)
        assert infos[rid]["iters"] == alone.iters
        assert np.array_equal(host(sv.result(rid)), host(alone.value)), (inst.M, kind, bc)
    sv.close()


def fno_net(seed, scale):
    """A neural operator with seeded random weights (spectral weights of size
    1/width, as in the FNO-G parity tests), output scale `scale`."""
    import torch
    from oracle import fno as ofno
    from paper_2404_02521_amd.fno import Fno
    rng = np.random.default_rng(seed)
    p = ofno.init_params(rng)
    for l in range(ofno.N_LAYERS):
        for k in ("Rr", "Ri"):
            p[f"{k}{l}"] = rng.normal(0.0, 1.0 / ofno.WIDTH, size=p[f"{k}{l}"].shape)
    net = Fno(max_batch=1, out_scale=scale, base=1)
    net.set_params(torch.from_numpy(ofno.flatten(p).astype(np.float32)).cuda())
    return net


@pytest.mark.parametrize("ragged", [False, True])
def test_fno_requests(pr, ragged):
    """PR_G_FNO requests through the server with an attached operator, mixed with
    a LOD request: refused (PR_EMODEL) before the operator is attached, the
    operator cannot be replaced while they wait, and each result equals the
    request solved alone with the same operator (status, K, fallback, value
    bitwise), with the fallback allowed and with PR_FLAG_NO_FALLBACK and tol 0
    (K = N)."""
    from paper_2404_02521_amd.serve import Server
    inst = plain_at_scale(1, M=129, n_slices=8, coarse_M=33)
    net = fno_net(7, inst.T / inst.n_slices)
    say("fno requests", "ragged" if ragged else "")
    sv = Server(2 << 30, max_resident=4, n_streams=3, ragged=ragged)
    with pytest.raises(pr.PararealError) as e:
        sv.submit(inst, pr.PR_G_FNO)
    assert e.value.status == pr._lib.PR_EMODEL
    sv.attach_fno(net)
    reqs = [(inst, pr.PR_G_FNO, 0),
            (inst.replace(tol=0.0), pr.PR_G_FNO, pr.PR_FLAG_NO_FALLBACK),
            (plain_at_scale(3, M=129, n_slices=8, coarse_M=33), pr.PR_G_LOD, 0),
            (plain_at_scale(4, M=97, n_slices=8, coarse_M=33), pr.PR_G_FNO, 0)]
    ids = [sv.submit(i, k, flags=f) for i, k, f in reqs]
    with pytest.raises(pr.PararealError) as e:
        sv.attach_fno(None)
    assert e.value.status == pr._lib.PR_EINVAL
    infos = sv.drain(ids, timeout_s=300)
    for rid, (i, k, f) in zip(ids, reqs):
        s = pr.Solver(i, coarse_kind=k, flags=f)
        if k == pr.PR_G_FNO:
            s.attach_fno(net)
        alone = s.solve()
        print("K", alone.iters, "fallback", alone.stats["coarse_fallback"])
        assert infos[rid]["status"] == alone.status
        assert infos[rid]["iters"] == alone.iters
        assert infos[rid]["coarse_fallback"] == alone.stats["coarse_fallback"]
        assert np.array_equal(host(sv.result(rid)), host(alone.value)), (i.M, k, f)
        s.close()
    assert infos[ids[1]]["iters"] == inst.n_slices
    sv.attach_fno(None)   # nothing waits for it any more
    sv.close()
    net.close()


def test_fno_request_falls_back_to_lod(pr):
    """A diverging operator (output scale 1e30: the first increment is not
    finite): the request restarts on LOD G and its result equals a LOD solve
    with 4 steps per slice, bitwise; with PR_FLAG_NO_FALLBACK it ends with
    PR_ENONFINITE."""
    from paper_2404_02521_amd.serve import Server
    inst = plain_at_scale(1, M=129, n_slices=8, coarse_M=33)
    net = fno_net(8, 1e30)
    say("fno request fallback")
    sv = Server(2 << 30, max_resident=2, n_streams=2)
    sv.attach_fno(net)
    ids = [sv.submit(inst, pr.PR_G_FNO), sv.submit(inst, pr.PR_G_FNO,
                                                   flags=pr.PR_FLAG_NO_FALLBACK)]
    infos = sv.drain(ids, timeout_s=300)
    lod = pr.Solver(inst.replace(coarse_steps_per_slice=4), coarse_kind=pr.PR_G_LOD)
    ref = lod.solve()
    assert infos[ids[0]]["status"] == 0 and infos[ids[0]]["coarse_fallback"] == 1
    assert infos[ids[0]]["iters"] == ref.iters
    assert np.array_equal(host(sv.result(ids[0])), host(ref.value))
    assert infos[ids[1]]["status"] == pr._lib.PR_ENONFINITE
    assert infos[ids[1]]["coarse_fallback"] == 0
    lod.close()
    sv.close()
    net.close()


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


@pytest.mark.parametrize("ragged", [False, True])
def test_served_requests_vs_oracle(pr, ragged):
    """Requests of the serving draw (129^2, N in {16, 32, 64}, T ~ U[0.25, 2],
    FP32 F), served in a mix with LOD and numerical coarse propagators: each
    result within 1e-5 relative of the oracle's FP64 serial F (the Parareal
    stop is 1e-7 relative)."""
    from paper_2404_02521_amd.serve import Server
    _, insts = serving_requests(1.0, 4, seed=21, sides=(129,))
    kinds = [pr.PR_G_LOD, pr.PR_G_NUMERICAL, pr.PR_G_LOD, pr.PR_G_NUMERICAL]
    say("served vs oracle", [(i.n_slices, round(i.T, 3)) for i in insts])
    sv = Server(4 << 30, max_resident=4, n_streams=2, ragged=ragged)
    ids = [sv.submit(inst, k) for inst, k in zip(insts, kinds)]
    infos = sv.drain(ids, timeout_s=300)
    for rid, inst in zip(ids, insts):
        assert infos[rid]["status"] == 0
        mf, _, _, _ = pr.plan(inst)
        ref = oracle.serial_fine(oproblem(inst), inst.n_slices, inst.T, mf)
        err = rel_max(host(sv.result(rid)), ref)
        print("N", inst.n_slices, "T %.3f" % inst.T, "K", infos[rid]["iters"], "err %.2e" % err)
        assert err <= 1e-5
    sv.close()


def test_bounded_queue_refuses_and_recovers(pr):
    """max_queued = 2: of six submissions made before the scheduler runs, two
    wait and four are refused with PR_EBUSY (counted); the two served results
    equal their solves alone, and after the drain the queue accepts again."""
    from paper_2404_02521_amd.serve import Server
    reqs = [plain_at_scale(400 + k, M=65, n_slices=8, coarse_M=33) for k in range(6)]
    say("bounded queue")
    sv = Server(1 << 30, max_resident=1, n_streams=1, max_queued=2)
    ids = [sv.submit(inst) for inst in reqs]
    assert [i is not None for i in ids] == [True, True, False, False, False, False]
    assert sv.rejected() == 4
    infos = sv.drain([i for i in ids if i is not None], timeout_s=120)
    for rid, inst in zip(ids[:2], reqs[:2]):
        assert infos[rid]["status"] == 0
        alone = pr.Solver(inst, coarse_kind=pr.PR_G_LOD).solve()
        assert np.array_equal(host(sv.result(rid)), host(alone.value))
    rid = sv.submit(reqs[2])
    assert rid is not None
    assert sv.drain([rid], timeout_s=120)[rid]["status"] == 0
    assert sv.rejected() == 4
    sv.close()
