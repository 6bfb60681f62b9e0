"""The neural coarse propagator inside the solver (PR_G_FNO) against an oracle
composition of the same definition: G(u) = B(tau1) + P_s(w + s * FNO(w)),
w = R_s(u - B(tau0)), with the DST-I transfers, the Coons patch and the FNO of
oracle.fno.  FP32 inference over FP64 transfers: within 1e-6 relative."""
import numpy as np
import pytest

import oracle
from helpers import oproblem, rel_max, say
from oracle import fno as ofno
from synthetic import plain_at_scale

pytestmark = pytest.mark.gpu


def gparams(seed):
    rng = np.random.default_rng(seed)
    p = ofno.init_params(rng)
    for l in range(ofno.N_LAYERS):
        for k in ("Rr", "Ri"):
            p[f"{k}{l}"] = rng.normal(0.0, 1.0 / ofno.WIDTH, size=p[f"{k}{l}"].shape)
    flat = ofno.flatten(p).astype(np.float32)
    return ofno.unflatten(flat.astype(np.float64)), flat


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def restrict_ref(pf, u, tau):
    ring = oracle.set_boundary(pf, tau, u)
    B = ofno.coons(ring, pf.M)
    w = (u - B)[1:-1, 1:-1]
    R = ofno.sine_restrict_matrix(pf.M - 2, 62)
    return R @ w @ R.T


def lod_base_ref(pf, wc, tau0, tau1, m=4):
    """The 64 x 64 grid's own LOD step from B(tau0) + wc, minus B(tau1)."""
    pc = pf.with_M(64)
    z = np.zeros((64, 64))
    B0 = ofno.coons(oracle.set_boundary(pc, tau0, z), 64)
    B1 = ofno.coons(oracle.set_boundary(pc, tau1, z), 64)
    v0 = B0.copy()
    v0[1:-1, 1:-1] += wc
    v1 = oracle.lod(pc, m, (tau1 - tau0) / m, tau0, v0)
    return (v1 - B1)[1:-1, 1:-1]


def g_ref(pf, p, u, tau0, tau1, scale, base="identity"):
    wc = restrict_ref(pf, u, tau0)
    inp = np.zeros((1, 64, 64, ofno.C_IN))
    inp[0, 1:-1, 1:-1, 0] = wc.astype(np.float32)
    inp[..., 1:5] = np.array([pf.sigma1, pf.sigma2, pf.rho, pf.r], dtype=np.float32)
    i = np.arange(64) / 63.0
    inp[..., 5] = i[None, :, None]
    inp[..., 6] = i[None, None, :]
    out = ofno.forward(p, inp)[0]
    P = ofno.sine_prolong_matrix(62, pf.M - 2)
    if base == "fine_lod":
        V = oracle.lod(pf, 1, tau1 - tau0, tau0, u)
        V[1:-1, 1:-1] += P @ (scale * out[1:-1, 1:-1]) @ P.T
        return V
    b = {"identity": wc, "zero": 0.0, "lod": None}[base]
    if base == "lod":
        b = lod_base_ref(pf, wc, tau0, tau1)
    wo = b + scale * out[1:-1, 1:-1]
    ring1 = oracle.set_boundary(pf, tau1, np.zeros((pf.M, pf.M)))
    B1 = ofno.coons(ring1, pf.M)
    V = B1.copy()
    V[1:-1, 1:-1] += P @ wo @ P.T
    return V


@pytest.fixture(scope="module")
def pr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2404_02521_amd as pr_
    return pr_


BASES = {"zero": 0, "identity": 1, "lod": 2, "fine_lod": 3}


def make(pr, inst, flat, scale, base="identity", **kw):
    from paper_2404_02521_amd.fno import Fno
    net = Fno(max_batch=1, out_scale=scale, base=BASES[base])
    net.set_params(dev(flat))
    s = pr.Solver(inst, coarse_kind=pr.PR_G_FNO, **kw)
    s.attach_fno(net)
    return s, net


@pytest.mark.parametrize("M,slice_,base", [(129, 0, "identity"), (131, 3, "identity"),
                                           (129, 2, "lod"), (131, 0, "zero"),
                                           (129, 1, "fine_lod")])
def test_fno_g_vs_oracle(pr, M, slice_, base):
    inst = plain_at_scale(2, M=M, n_slices=8, coarse_M=33)
    pf = oproblem(inst)
    dT = inst.T / inst.n_slices
    p, flat = gparams(5)
    mf = oracle.steps_for(pf, dT, 0.9)
    u = oracle.fine(pf, mf, dT / mf, 0.0, oracle.payoff_grid(pf)) if slice_ else oracle.payoff_grid(pf)
    u = oracle.set_boundary(pf, slice_ * dT, u)
    say("fno G vs oracle", M, slice_, base)
    s, net = make(pr, inst, flat, dT, base)
    got = s.apply(pr.PR_OP_COARSE, slice_, dev(u)).cpu().numpy()
    ref = g_ref(pf, p, u, slice_ * dT, (slice_ + 1) * dT, dT, base)
    assert rel_max(got, ref) <= 1e-6
    s.close()
    net.close()


@pytest.mark.parametrize("base", ["identity", "lod", "fine_lod"])
def test_fno_pair_vs_oracle(pr, base):
    inst = plain_at_scale(4, M=129, n_slices=8, coarse_M=33)
    pf = oproblem(inst)
    dT = inst.T / inst.n_slices
    _, flat = gparams(6)
    mf = oracle.steps_for(pf, dT, 0.9)
    u0 = oracle.fine(pf, mf, dT / mf, 0.0, oracle.payoff_grid(pf))
    u1 = oracle.fine(pf, mf, dT / mf, dT, u0)
    say("fno pair vs oracle", base)
    s, net = make(pr, inst, flat, dT, base)
    got = s.fno_pair(1, dev(u0), dev(u1), BASES[base]).cpu().numpy()
    w0 = restrict_ref(pf, u0, dT)
    w1 = restrict_ref(pf, u1, 2 * dT)
    pc = pf.with_M(64)
    z = np.zeros((64, 64))
    B0 = ofno.coons(oracle.set_boundary(pc, dT, z), 64)
    B1 = ofno.coons(oracle.set_boundary(pc, 2 * dT, z), 64)
    pad = lambda a: np.pad(a, 1)
    b1 = B1 + (pad(lod_base_ref(pf, w0, dT, 2 * dT)) if base == "lod" else 0.0)
    if base == "fine_lod":
        b1 = B1 + pad(restrict_ref(pf, oracle.lod(pf, 1, dT, dT, u0), 2 * dT))
    ref = np.stack([pad(w0), b1, B0 + pad(w0), B1 + pad(w1)])
    for k in range(4):
        assert rel_max(got[k], ref[k]) <= 1e-6, k
    s.close()
    net.close()


def test_fno_parareal_finite_termination(pr):
    """With tol 0 the neural G still gives serial F exactly at K = N."""
    inst = plain_at_scale(1, M=129, n_slices=8, coarse_M=33).replace(tol=0.0)
    _, flat = gparams(7)
    say("fno parareal K=N")
    s, net = make(pr, inst, flat, inst.T / inst.n_slices, flags=pr.PR_FLAG_NO_FALLBACK)
    res = s.solve()
    assert res.iters == inst.n_slices and res.stats["coarse_fallback"] == 0
    assert np.array_equal(res.value.cpu().numpy(), s.serial_fine().value.cpu().numpy())
    s.close()
    net.close()


def test_fno_fallback_to_lod(pr):
    """A diverging neural G (output scale 1e30 makes the first increment
    non-finite) restarts with the LOD propagator: same result, bitwise, as a LOD
    solver with 4 steps per slice."""
    inst = plain_at_scale(1, M=129, n_slices=8, coarse_M=33)
    _, flat = gparams(8)
    say("fno fallback")
    s, net = make(pr, inst, flat, 1e30)
    res = s.solve()
    assert res.stats["coarse_fallback"] == 1
    lod = pr.Solver(inst.replace(coarse_steps_per_slice=4), coarse_kind=pr.PR_G_LOD)
    ref = lod.solve()
    assert res.iters == ref.iters
    assert np.array_equal(res.value.cpu().numpy(), ref.value.cpu().numpy())
    s.close()
    lod.close()
    net.close()


def test_nonfinite_increment_without_fallback(pr):
    """The same diverging neural G with PR_FLAG_NO_FALLBACK: the norm's
    non-finite flag ends the solve with PR_ENONFINITE after the first
    iteration, and the solver stays usable (its serial F is unchanged)."""
    inst = plain_at_scale(1, M=129, n_slices=8, coarse_M=33)
    _, flat = gparams(8)
    say("fno non-finite, no fallback")
    s, net = make(pr, inst, flat, 1e30, flags=pr.PR_FLAG_NO_FALLBACK)
    ser0 = s.serial_fine().value.cpu().numpy()
    with pytest.raises(pr.PararealError) as e:
        s.solve()
    assert e.value.status == pr._lib.PR_ENONFINITE
    assert np.array_equal(s.serial_fine().value.cpu().numpy(), ser0)
    s.close()
    net.close()


def test_fno_rejected_without_operator(pr):
    inst = plain_at_scale(1, M=129, n_slices=8, coarse_M=33)
    s = pr.Solver(inst, coarse_kind=pr.PR_G_FNO)
    with pytest.raises(pr.PararealError) as e:
        s.solve()
    assert e.value.status == pr._lib.PR_EMODEL
    s.close()
