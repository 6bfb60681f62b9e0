"""The GPU Fourier neural operator (pr_fno_*) against the NumPy FP64 oracle.

Bars: FP32 forward within 1e-5 (relative max-norm and relative L2), BF16
forward within 2e-2 relative L2; FP32 gradients within 1e-4 relative L2 per
parameter block, BF16 gradients with cosine >= 0.999 and relative L2 <= 2e-2
over the whole vector; the loss (evaluated in FP64 on FP32 inputs) within
1e-9 relative, its gradient within 1e-6; Adam within FP32 rounding.
"""
import numpy as np
import pytest

from helpers import rel_max, say
from oracle import fno as ofno
from synthetic import fno_batch, fno_pairs

pytestmark = pytest.mark.gpu

DT = 1.0 / 64


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_02521_amd import fno
    return fno


def test_params(seed):
    """Initial weights of the oracle, with spectral multipliers of the size of the
    pointwise path so that every block shapes the output."""
    rng = np.random.default_rng(seed)
    p = ofno.init_params(rng)
    for l in range(ofno.N_LAYERS):
        for k in ("Rr", "Ri"):
            p[f"{k}{l}"] = rng.normal(0.0, 1.0 / ofno.WIDTH, size=p[f"{k}{l}"].shape)
    flat = ofno.flatten(p).astype(np.float32)
    return ofno.unflatten(flat.astype(np.float64)), flat


test_params.__test__ = False


def oracle_input(w, meta):
    B = w.shape[0]
    inp = np.zeros((B, 64, 64, ofno.C_IN))
    inp[..., 0] = w
    inp[..., 1:5] = meta[:, None, None, :]
    i = np.arange(64) / 63.0
    inp[..., 5] = i[None, :, None]
    inp[..., 6] = i[None, None, :]
    return inp


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cosine(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_param_count(F):
    assert F.param_count() == ofno.flatten(ofno.init_params(np.random.default_rng(0))).size


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_forward_vs_oracle(F, prec):
    from paper_2404_02521_amd import _lib as L
    p, flat = test_params(0)
    w, meta = fno_batch(10, 3)
    say("fno forward", prec)
    net = F.Fno(max_batch=4)
    net.set_params(dev(flat))
    out = net.forward(dev(w), dev(meta), L.PR_FNO_FP32 if prec == "fp32" else L.PR_FNO_BF16)
    got = out.cpu().numpy()
    ref = ofno.forward(p, oracle_input(w.astype(np.float64), meta.astype(np.float64)))
    if prec == "fp32":
        assert rel_max(got, ref) <= 1e-5
        assert rel_l2(got, ref) <= 1e-5
    else:
        assert rel_l2(got, ref) <= 2e-2
    net.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_backward_vs_oracle(F, prec):
    from paper_2404_02521_amd import _lib as L
    p, flat = test_params(1)
    w, meta = fno_batch(11, 2)
    gout = np.random.default_rng(12).normal(size=(2, 64, 64)).astype(np.float32)
    say("fno backward", prec)
    net = F.Fno(max_batch=2)
    net.set_params(dev(flat))
    net.forward(dev(w), dev(meta), L.PR_FNO_FP32 if prec == "fp32" else L.PR_FNO_BF16)
    net.backward(dev(gout))
    g = net.grads().cpu().numpy()
    _, cache = ofno.forward(p, oracle_input(w.astype(np.float64), meta.astype(np.float64)),
                            keep=True)
    gref = ofno.flatten(ofno.backward(p, cache, gout.astype(np.float64)))
    if prec == "fp32":
        o = 0
        for name, shape in ofno.param_shapes():
            n = int(np.prod(shape))
            assert rel_l2(g[o:o + n], gref[o:o + n]) <= 1e-4, name
            o += n
    else:
        assert cosine(g, gref) >= 0.999
        assert rel_l2(g, gref) <= 2e-2
    net.close()


@pytest.mark.parametrize("lam,scale", [(1.0, 1.0), (0.5, 1.0 / 64)])
def test_loss_vs_oracle(F, lam, scale):
    pairs, meta = fno_pairs(20, 3)
    pred = (np.random.default_rng(21).normal(size=(3, 64, 64)) * 0.05).astype(np.float32)
    say("fno loss", lam, scale)
    net = F.Fno(max_batch=3)
    (lo, data, res), g = net.loss(dev(pred), dev(pairs), dev(meta), DT, lam, scale)
    P = pairs.astype(np.float64)
    ref, gref = ofno.loss(scale * pred.astype(np.float64), P[:, 0], P[:, 1], P[:, 2], P[:, 3],
                          meta.astype(np.float64), DT, lam)
    assert abs(lo - ref) <= 1e-9 * abs(ref)
    assert rel_max(g.cpu().numpy(), scale * gref) <= 1e-6
    net.close()


def test_loss_residual_vanishes_on_eigenfunction(F):
    """Q = i j is an eigenfunction of the index-form operator with eigenvalue
    lambda = rho s1 s2 + r; V_in = Q, V1 = Q (1 + dT lambda/2) / (1 - dT lambda/2)
    makes the Crank-Nicolson residual zero."""
    s1, s2, rho, r = 0.3, 0.2, 0.5, 0.05
    lam_ab = rho * s1 * s2 + 2 * r - r
    f = (1 + DT * lam_ab / 2) / (1 - DT * lam_ab / 2)
    i = np.arange(64.0)
    Q = np.outer(i, i)
    pairs = np.zeros((1, 4, 64, 64))
    pairs[0, 1] = f * Q
    pairs[0, 2] = Q
    pairs[0, 3] = f * Q
    meta = np.array([[s1, s2, rho, r]], dtype=np.float32)
    say("fno residual eigenfunction")
    net = F.Fno(max_batch=1)
    (lo, data, res), _ = net.loss(dev(np.zeros((1, 64, 64), np.float32)),
                                  dev(pairs.astype(np.float32)), dev(meta), DT, 1.0)
    assert res <= 1e-10 * float((Q[1:-1, 1:-1] ** 2).mean())
    net.close()


def test_adam_vs_oracle(F):
    from paper_2404_02521_amd import _lib as L
    p, flat = test_params(2)
    w, meta = fno_batch(13, 2)
    say("fno adam")
    net = F.Fno(max_batch=2)
    net.set_params(dev(flat))
    P = {k: v.copy() for k, v in ofno.unflatten(flat.astype(np.float64)).items()}
    m = {k: np.zeros_like(v) for k, v in P.items()}
    v = {k: np.zeros_like(v) for k, v in P.items()}
    rng = np.random.default_rng(14)
    for step in (1, 2, 3):
        gout = rng.normal(size=(2, 64, 64)).astype(np.float32)
        net.forward(dev(w), dev(meta), L.PR_FNO_FP32)
        net.backward(dev(gout))
        g = ofno.unflatten(net.grads().cpu().numpy().astype(np.float64))
        net.adam(1e-3, step)
        ofno.adam(P, g, m, v, step, 1e-3)
        got = net.params().cpu().numpy()
        assert np.allclose(got, ofno.flatten(P), rtol=1e-6, atol=2e-7), step
    net.close()


def test_train_step_equals_its_parts(F):
    """pr_fno_train_step on gathered pairs = forward + loss + backward + Adam, bitwise."""
    import torch
    from paper_2404_02521_amd import _lib as L
    _, flat = test_params(3)
    pairs, meta = fno_pairs(30, 6)
    idx = np.array([4, 1, 3], dtype=np.int32)
    say("fno train step")
    a = F.Fno(max_batch=3, out_scale=DT)
    a.set_params(dev(flat))
    loss_a = a.train_step(dev(pairs), dev(meta), dev(idx), DT, 1e-3, 1, L.PR_FNO_BF16)
    pa = a.params().cpu().numpy()
    b = F.Fno(max_batch=3, out_scale=DT)
    b.set_params(dev(flat))
    sel = dev(pairs[idx])
    out = b.forward(sel[:, 0].contiguous(), dev(meta[idx]), L.PR_FNO_BF16)
    (lo, _, _), g = b.loss(out, sel, dev(meta[idx]), DT, 1.0, DT)
    b.backward(g)
    b.adam(1e-3, 1)
    pb = b.params().cpu().numpy()
    assert loss_a[0] == lo
    assert np.array_equal(pa, pb)
    assert not np.array_equal(pa, flat)
    a.close()
    b.close()
    torch.cuda.synchronize()
