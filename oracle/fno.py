"""Fourier neural operator coarse propagator in NumPy FP64 (TEST INFRASTRUCTURE ONLY).

Follows Sec. 3.4 (FNO: lifting, Fourier layers of truncated-mode multipliers
plus a pointwise path, projection) and Sec. 3.5 (physics-informed loss), with
the sizes used here: width 32, four Fourier layers, 12 x 12 retained modes
on a 64 x 64 grid, GELU, two-layer lift (C_in -> 64 -> 32) and projection
(32 -> 128 -> 1).  Gradients are derived by hand and pinned against central
differences in the tests.

Definitions (v has shape (B, 64, 64, C): batch, x index, y index, channel):
  modes   kx in {0..11, -12..-1} (24), ky in {0..11} (12)
  DFT     X[b,k,q,c] = sum_{x,y} v[b,x,y,c] e^{-2 pi i (kx x + ky y)/64}
  mix     Y[b,k,q,o] = sum_i X[b,k,q,i] R[k,q,i,o]        (complex R)
  inverse u[b,x,y,o] = Re sum_{k,q} c_q Y[b,k,q,o] e^{+2 pi i (kx x + ky y)/64} / 4096,
          c_0 = 1, c_q = 2 for q >= 1 (the conjugate half of the spectrum)
  layer   v' = act(u + v W + b), act = GELU (exact erf form) except after the last
  network out = (GELU(GELU(in L1 + l1) L2 + l2 ... ) ...): lift, 4 layers, project
The network maps the channels [w, s1, s2, rho, r, x/S, y/S] of one sample to
the change of w over one slice; the coarse state after the slice is w + out.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

N_GRID = 64
MX, MY = 12, 12
KX = np.array(list(range(MX)) + list(range(-MX, 0)))
KY = np.arange(MY)
WIDTH = 32
N_LAYERS = 4
LIFT_H = 64
PROJ_H = 128
C_IN = 7


def param_shapes(cin=C_IN, width=WIDTH, layers=N_LAYERS):
    """Ordered parameter list (name, shape); R is stored as real and imaginary parts."""
    s = [("L1", (cin, LIFT_H)), ("l1", (LIFT_H,)), ("L2", (LIFT_H, width)), ("l2", (width,))]
    for l in range(layers):
        s += [(f"Rr{l}", (len(KX), MY, width, width)), (f"Ri{l}", (len(KX), MY, width, width)),
              (f"W{l}", (width, width)), (f"b{l}", (width,))]
    s += [("P1", (width, PROJ_H)), ("p1", (PROJ_H,)), ("P2", (PROJ_H, 1)), ("p2", (1,))]
    return s


def init_params(rng, cin=C_IN, width=WIDTH, layers=N_LAYERS):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for the dense layers; spectral weights
    uniform with scale 1/(width*width) (the usual FNO initialisation)."""
    p = {}
    for name, shape in param_shapes(cin, width, layers):
        if name.startswith(("Rr", "Ri")):
            p[name] = rng.uniform(0.0, 1.0, size=shape) / (width * width)
        elif len(shape) == 2:
            bound = 1.0 / math.sqrt(shape[0])
            p[name] = rng.uniform(-bound, bound, size=shape)
        else:
            fan = {"l1": cin, "l2": LIFT_H, "p1": width, "p2": PROJ_H}.get(name, width)
            bound = 1.0 / math.sqrt(fan)
            p[name] = rng.uniform(-bound, bound, size=shape)
    return p


def flatten(p, cin=C_IN, width=WIDTH, layers=N_LAYERS):
    return np.concatenate([np.asarray(p[n], dtype=np.float64).ravel()
                           for n, _ in param_shapes(cin, width, layers)])


def unflatten(flat, cin=C_IN, width=WIDTH, layers=N_LAYERS):
    p, o = {}, 0
    for n, shape in param_shapes(cin, width, layers):
        k = int(np.prod(shape))
        p[n] = flat[o:o + k].reshape(shape).copy()
        o += k
    assert o == flat.size
    return p


def dft_matrices():
    x = np.arange(N_GRID)
    Fx = np.exp(-2j * np.pi * np.outer(KX, x) / N_GRID)            # (24, 64)
    Fy = np.exp(-2j * np.pi * np.outer(x, KY) / N_GRID)            # (64, 12)
    c = np.where(KY == 0, 1.0, 2.0)
    Gx = np.exp(2j * np.pi * np.outer(x, KX) / N_GRID)             # (64, 24)
    Gy = (c[:, None] * np.exp(2j * np.pi * np.outer(KY, x) / N_GRID)) / (N_GRID * N_GRID)  # (12, 64)
    return Fx, Fy, Gx, Gy


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def spectral(v, Rr, Ri, mats):
    Fx, Fy, Gx, Gy = mats
    X = np.einsum("kx,bxyc,yq->bkqc", Fx, v, Fy)
    R = Rr + 1j * Ri
    Y = np.einsum("bkqi,kqio->bkqo", X, R)
    u = np.einsum("xk,bkqo,qy->bxyo", Gx, Y, Gy).real
    return u, X, Y


def spectral_backward(gu, X, Rr, Ri, mats):
    Fx, Fy, Gx, Gy = mats
    gY = np.einsum("xk,bxyo,qy->bkqo", Gx.conj(), gu, Gy.conj())
    R = Rr + 1j * Ri
    gX = np.einsum("bkqo,kqio->bkqi", gY, R.conj())
    gR = np.einsum("bkqi,bkqo->kqio", X.conj(), gY)
    gv = np.einsum("kx,bkqc,yq->bxyc", Fx.conj(), gX, Fy.conj()).real
    return gv, gR.real, gR.imag


def forward(p, inp, layers=N_LAYERS, keep=False):
    """inp: (B, 64, 64, C_in) -> out (B, 64, 64)."""
    mats = dft_matrices()
    cache = {"inp": inp}
    z1 = inp @ p["L1"] + p["l1"]
    h1 = gelu(z1)
    v = h1 @ p["L2"] + p["l2"]
    cache.update(z1=z1, h1=h1)
    vs, zs, Xs = [v], [], []
    for l in range(layers):
        u, X, _ = spectral(v, p[f"Rr{l}"], p[f"Ri{l}"], mats)
        z = u + v @ p[f"W{l}"] + p[f"b{l}"]
        v = gelu(z) if l < layers - 1 else z
        zs.append(z)
        Xs.append(X)
        vs.append(v)
    zq = v @ p["P1"] + p["p1"]
    hq = gelu(zq)
    out = (hq @ p["P2"] + p["p2"])[..., 0]
    cache.update(vs=vs, zs=zs, Xs=Xs, zq=zq, hq=hq)
    return (out, cache) if keep else out


def backward(p, cache, gout, layers=N_LAYERS):
    """gout = dL/dout (B, 64, 64) -> dict of parameter gradients (same keys as p)."""
    mats = dft_matrices()
    g = {}
    go = gout[..., None]
    hq = cache["hq"]
    g["P2"] = np.einsum("bxyh,bxyo->ho", hq, go)
    g["p2"] = go.sum(axis=(0, 1, 2))
    gzq = (go @ p["P2"].T) * gelu_grad(cache["zq"])
    v = cache["vs"][layers]
    g["P1"] = np.einsum("bxyc,bxyh->ch", v, gzq)
    g["p1"] = gzq.sum(axis=(0, 1, 2))
    gv = gzq @ p["P1"].T
    for l in reversed(range(layers)):
        z = cache["zs"][l]
        gz = gv * gelu_grad(z) if l < layers - 1 else gv
        vin = cache["vs"][l]
        g[f"W{l}"] = np.einsum("bxyi,bxyo->io", vin, gz)
        g[f"b{l}"] = gz.sum(axis=(0, 1, 2))
        gvs, g[f"Rr{l}"], g[f"Ri{l}"] = spectral_backward(gz, cache["Xs"][l], p[f"Rr{l}"],
                                                          p[f"Ri{l}"], mats)
        gv = gvs + gz @ p[f"W{l}"].T
    g["L2"] = np.einsum("bxyh,bxyc->hc", cache["h1"], gv)
    g["l2"] = gv.sum(axis=(0, 1, 2))
    gz1 = (gv @ p["L2"].T) * gelu_grad(cache["z1"])
    g["L1"] = np.einsum("bxyi,bxyh->ih", cache["inp"], gz1)
    g["l1"] = gz1.sum(axis=(0, 1, 2))
    return g


# --------------------------------------------------------------------------- loss
def lh_interior(w, s1, s2, rho, r):
    """The operator of Eq. (fd) in index form on the interior of a 64 x 64 grid
    (w: (B, 64, 64); parameters per sample, shape (B,))."""
    i = np.arange(N_GRID, dtype=np.float64)
    I = i[1:-1][None, :, None]
    J = i[1:-1][None, None, :]
    a = (0.5 * s1 * s1)[:, None, None] * I * I
    b = (0.5 * s2 * s2)[:, None, None] * J * J
    g = (0.25 * rho * s1 * s2)[:, None, None] * I * J
    hr = (0.5 * r)[:, None, None]
    c = w[:, 1:-1, 1:-1]
    uxx = w[:, 2:, 1:-1] - 2 * c + w[:, :-2, 1:-1]
    uyy = w[:, 1:-1, 2:] - 2 * c + w[:, 1:-1, :-2]
    uxy = w[:, 2:, 2:] + w[:, :-2, :-2] - w[:, 2:, :-2] - w[:, :-2, 2:]
    ux = w[:, 2:, 1:-1] - w[:, :-2, 1:-1]
    uy = w[:, 1:-1, 2:] - w[:, 1:-1, :-2]
    return a * uxx + b * uyy + g * uxy + hr * I * ux + hr * J * uy - r[:, None, None] * c


def ring_mask():
    m = np.zeros((N_GRID, N_GRID))
    m[1:-1, 1:-1] = 1.0
    return m


def loss(pred, w_in, B1, V_in, V_tgt, meta, dT, lam=1.0):
    """Data MSE + lam * mean(R^2) on the 64^2 interior, with
    V1 = B1 + w_in + pred (ring of pred ignored: the ring is the Dirichlet data)
    and the Crank-Nicolson residual R = (V1 - V_in) - dT L_h((V1 + V_in)/2) of the
    PDE (the PDE-residual term of Sec. 3.5, on the grid).  All arrays (B, 64, 64);
    meta (B, 4) = s1, s2, rho, r.  Returns (loss, dL/dpred)."""
    B = pred.shape[0]
    V1 = B1 + w_in + pred * ring_mask()
    n_int = (N_GRID - 2) ** 2
    d = V1 - V_tgt
    data = float((d[:, 1:-1, 1:-1] ** 2).sum()) / (B * n_int)
    s1, s2, rho, r = (meta[:, k] for k in range(4))
    R = (V1 - V_in)[:, 1:-1, 1:-1] - dT * lh_interior(0.5 * (V1 + V_in), s1, s2, rho, r)
    res = float((R ** 2).sum()) / (B * n_int)
    g = np.zeros_like(pred)
    g[:, 1:-1, 1:-1] += 2.0 * d[:, 1:-1, 1:-1] / (B * n_int)
    gR = lam * 2.0 * R / (B * n_int)
    g[:, 1:-1, 1:-1] += gR
    # adjoint of -dT * L_h(0.5 * V1): scatter gR through the 9-point stencil
    gw = np.zeros_like(pred)
    i = np.arange(N_GRID, dtype=np.float64)
    I = i[1:-1][None, :, None]
    J = i[1:-1][None, None, :]
    a = (0.5 * s1 * s1)[:, None, None] * I * I
    b = (0.5 * s2 * s2)[:, None, None] * J * J
    gg = (0.25 * rho * s1 * s2)[:, None, None] * I * J
    hr = (0.5 * r)[:, None, None]
    cc = -0.5 * dT * gR
    gw[:, 1:-1, 1:-1] += cc * (-2 * a - 2 * b - r[:, None, None])
    gw[:, 2:, 1:-1] += cc * (a + hr * I)
    gw[:, :-2, 1:-1] += cc * (a - hr * I)
    gw[:, 1:-1, 2:] += cc * (b + hr * J)
    gw[:, 1:-1, :-2] += cc * (b - hr * J)
    gw[:, 2:, 2:] += cc * gg
    gw[:, :-2, :-2] += cc * gg
    gw[:, 2:, :-2] -= cc * gg
    gw[:, :-2, 2:] -= cc * gg
    g += gw
    return data + lam * res, g * ring_mask()


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) in place; step counts from 1."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def lr_at(epoch, lr0=1e-3, decay=0.96, every=25):
    """Step decay of Sec. 3.5: 0.96 every 25 epochs from 1e-3."""
    return lr0 * decay ** (epoch // every)


# ------------------------------------------------------------ spectral transfer
def sine_restrict_matrix(nf, nc):
    """DST-I restriction between interior node sets of nf and nc points:
    coefficients a_k = 2/(nf+1) sum_i w_i sin(pi k i/(nf+1)), k = 1..nc, then
    w_c[i] = sum_k a_k sin(pi k i/(nc+1)).  Shape (nc, nf)."""
    k = np.arange(1, nc + 1)
    i_f = np.arange(1, nf + 1)
    i_c = np.arange(1, nc + 1)
    Sf = (2.0 / (nf + 1)) * np.sin(np.pi * np.outer(k, i_f) / (nf + 1))   # (nc, nf)
    Sc = np.sin(np.pi * np.outer(i_c, k) / (nc + 1))                      # (nc, nc)
    return Sc @ Sf


def sine_prolong_matrix(nc, nf):
    """Zero-padded DST-I prolongation, shape (nf, nc)."""
    k = np.arange(1, nc + 1)
    i_c = np.arange(1, nc + 1)
    i_f = np.arange(1, nf + 1)
    Sc = (2.0 / (nc + 1)) * np.sin(np.pi * np.outer(k, i_c) / (nc + 1))   # (nc, nc)
    Sf = np.sin(np.pi * np.outer(i_f, k) / (nf + 1))                      # (nf, nc)
    return Sf @ Sc


def coons(ring, M):
    """Transfinite (Coons) interpolation of the ring values of an M x M grid."""
    t = np.linspace(0.0, 1.0, M)
    xi, eta = t[:, None], t[None, :]
    B = ((1 - xi) * ring[0:1, :] + xi * ring[-1:, :] + (1 - eta) * ring[:, 0:1]
         + eta * ring[:, -1:]
         - ((1 - xi) * (1 - eta) * ring[0, 0] + xi * (1 - eta) * ring[-1, 0]
            + (1 - xi) * eta * ring[0, -1] + xi * eta * ring[-1, -1]))
    return B
