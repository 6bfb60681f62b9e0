"""Pins of the NumPy FNO oracle: DFT conventions against numpy.fft, hand-derived
gradients against central differences (FP64), special cases, transfers."""
import numpy as np
import pytest

from oracle import fno


def small_params(rng, width=4, layers=2, cin=3):
    p = {}
    for name, shape in fno.param_shapes(cin, width, layers):
        p[name] = rng.standard_normal(shape) * (0.05 if name.startswith("R") else 0.3)
    return p


def test_dft_matches_numpy_fft():
    rng = np.random.default_rng(0)
    v = rng.standard_normal((2, 64, 64, 3))
    Fx, Fy, Gx, Gy = fno.dft_matrices()
    X = np.einsum("kx,bxyc,yq->bkqc", Fx, v, Fy)
    ref = np.fft.fft2(v, axes=(1, 2))[:, fno.KX % 64][:, :, fno.KY]
    assert np.abs(X - ref).max() < 1e-10
    # the inverse with all retained modes of a field built from those modes is exact
    spec = np.zeros((64, 33), dtype=complex)
    for k in fno.KX:
        for q in fno.KY:
            spec[k % 64, q] = rng.standard_normal() + 1j * rng.standard_normal()
    # the ky = 0 column of a real field is Hermitian in kx; kx = -12 has no retained
    # partner (+12 is cut), so it must be zero there for the field to be representable
    spec[0, 0] = spec[0, 0].real
    spec[(-12) % 64, 0] = 0.0
    for k in range(1, 12):
        spec[(-k) % 64, 0] = np.conj(spec[k, 0])
    field = np.fft.irfft2(spec, s=(64, 64))
    Xf = np.einsum("kx,xy,yq->kq", Fx, field, Fy)
    back = np.einsum("xk,kq,qy->xy", Gx, Xf, Gy).real
    assert np.abs(back - field).max() < 1e-12


def test_identity_spectral_weights_reproduce_low_modes():
    """R = identity per mode -> the layer's spectral part is the mode truncation."""
    rng = np.random.default_rng(1)
    v = rng.standard_normal((1, 64, 64, 2))
    Rr = np.broadcast_to(np.eye(2), (24, 12, 2, 2)).copy()
    u, _, _ = fno.spectral(v, Rr, np.zeros_like(Rr), fno.dft_matrices())
    F = np.fft.fft2(v[0, :, :, 0])
    keep = np.zeros((64, 64))
    for k in fno.KX:
        for q in fno.KY:
            keep[k % 64, q] = 1.0
            keep[(-k) % 64, (-q) % 64] = 1.0
    # Re(.) of the unpaired mode (-12, 0) keeps half of it and half of its conjugate (+12, 0)
    keep[(-12) % 64, 0] = keep[12, 0] = 0.5
    ref = np.fft.ifft2(keep * F).real
    assert np.abs(u[0, :, :, 0] - ref).max() < 1e-12


def test_zero_spectral_identity_pointwise_is_gelu():
    """Zero spectral weights, identity W, zero bias: one hidden layer is pointwise GELU."""
    rng = np.random.default_rng(2)
    p = small_params(rng, width=3, layers=2, cin=3)
    for l in range(2):
        p[f"Rr{l}"][:] = 0
        p[f"Ri{l}"][:] = 0
        p[f"W{l}"] = np.eye(3)
        p[f"b{l}"][:] = 0
    inp = rng.standard_normal((1, 64, 64, 3))
    out, cache = fno.forward(p, inp, layers=2, keep=True)
    v0 = cache["vs"][0]
    assert np.allclose(cache["vs"][1], fno.gelu(v0), atol=1e-14)
    assert np.allclose(cache["vs"][2], fno.gelu(v0), atol=1e-14)   # last layer: no activation


@pytest.mark.parametrize("name", ["L1", "l1", "L2", "Rr0", "Ri0", "W0", "b0", "Rr1", "Ri1",
                                  "W1", "b1", "P1", "p1", "P2", "p2"])
def test_gradients_central_differences(name):
    rng = np.random.default_rng(3)
    p = small_params(rng, width=4, layers=2, cin=3)
    inp = rng.standard_normal((1, 64, 64, 3))
    gout = rng.standard_normal((1, 64, 64))
    out, cache = fno.forward(p, inp, layers=2, keep=True)
    g = fno.backward(p, cache, gout, layers=2)
    L = lambda q: float((fno.forward(q, inp, layers=2) * gout).sum())
    flat = p[name].ravel()
    idx = rng.choice(flat.size, size=min(4, flat.size), replace=False)
    eps = 1e-6
    for i in idx:
        qp = {k: v.copy() for k, v in p.items()}
        qm = {k: v.copy() for k, v in p.items()}
        qp[name].ravel()[i] += eps
        qm[name].ravel()[i] -= eps
        fd = (L(qp) - L(qm)) / (2 * eps)
        an = g[name].ravel()[i]
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, i, fd, an)


def test_loss_gradient_central_differences():
    rng = np.random.default_rng(4)
    B = 2
    pred = rng.standard_normal((B, 64, 64)) * 0.01
    w_in = rng.standard_normal((B, 64, 64)) * 0.1
    B1 = rng.standard_normal((B, 64, 64))
    V_in = rng.standard_normal((B, 64, 64))
    V_t = rng.standard_normal((B, 64, 64))
    meta = np.array([[0.3, 0.2, 0.5, 0.05], [0.4, 0.25, -0.3, 0.08]])
    L0, g = fno.loss(pred, w_in, B1, V_in, V_t, meta, 1.0 / 64, lam=0.7)
    for (b, i, j) in [(0, 1, 1), (1, 20, 33), (0, 62, 62), (1, 0, 5), (0, 31, 1)]:
        e = np.zeros_like(pred)
        e[b, i, j] = 1e-6
        fd = (fno.loss(pred + e, w_in, B1, V_in, V_t, meta, 1.0 / 64, 0.7)[0]
              - fno.loss(pred - e, w_in, B1, V_in, V_t, meta, 1.0 / 64, 0.7)[0]) / 2e-6
        assert abs(fd - g[b, i, j]) <= 1e-6 * max(1.0, abs(fd)), (b, i, j, fd, g[b, i, j])


def test_residual_vanishes_on_monomial_eigenfunction():
    """For an eigenfunction Q of L_h with eigenvalue lam, V1 = (1+dT lam/2)/(1-dT lam/2) Q
    solves the Crank-Nicolson relation exactly: zero PDE residual."""
    x = np.arange(64) * (4.0 / 63)
    s1, s2, rho, r = 0.3, 0.2, 0.5, 0.05
    Q = np.outer(x, x)[None]                      # x*y: lam = rho s1 s2 + r
    lam = rho * s1 * s2 + r
    dT = 1.0 / 64
    V1 = (1 + dT * lam / 2) / (1 - dT * lam / 2) * Q
    meta = np.array([[s1, s2, rho, r]])
    L, _ = fno.loss(np.zeros_like(Q), Q, V1 - Q, Q, V1, meta, dT, lam=1.0)
    assert L < 1e-26


def test_sine_transfer_identities():
    Rs = fno.sine_restrict_matrix(511, 62)
    Ps = fno.sine_prolong_matrix(62, 511)
    assert np.abs(Rs @ Ps - np.eye(62)).max() < 1e-12
    # a single sine mode restricts to the same mode
    i_f = np.arange(1, 512)
    i_c = np.arange(1, 63)
    for k in (1, 7, 62):
        assert np.abs(Rs @ np.sin(np.pi * k * i_f / 512) - np.sin(np.pi * k * i_c / 63)).max() < 1e-12
    # modes above the cut-off are removed
    assert np.abs(Rs @ np.sin(np.pi * 100 * i_f / 512)).max() < 1e-12


def test_coons_reproduces_ring_and_bilinear():
    M = 17
    t = np.linspace(0, 1, M)
    f = lambda a, b: 1.0 + 2 * a - 3 * b + 0.5 * a * b
    F = f(t[:, None], t[None, :])
    B = fno.coons(F, M)
    assert np.abs(B - F).max() < 1e-13
    G = np.sin(3 * t)[:, None] * np.cos(2 * t)[None, :]
    BG = fno.coons(G, M)
    assert np.abs(BG[0] - G[0]).max() < 1e-14 and np.abs(BG[:, -1] - G[:, -1]).max() < 1e-14


def test_adam_matches_definition():
    p = {"a": np.array([1.0, -2.0])}
    m = {"a": np.zeros(2)}
    v = {"a": np.zeros(2)}
    g = {"a": np.array([0.5, -0.25])}
    fno.adam(p, g, m, v, 1, 1e-3)
    # first step of Adam moves every coordinate by lr * sign(g) (bias-corrected)
    assert np.allclose(p["a"], [1.0 - 1e-3, -2.0 + 1e-3], atol=1e-9)
    assert fno.lr_at(0) == 1e-3 and abs(fno.lr_at(25) - 0.96e-3) < 1e-18 and abs(fno.lr_at(74) - 0.96 ** 2 * 1e-3) < 1e-18


def test_param_count():
    n = sum(int(np.prod(s)) for _, s in fno.param_shapes())
    assert 2_300_000 < n < 2_450_000
