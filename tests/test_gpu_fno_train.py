"""Training the neural coarse propagator on the GPU from trajectories of F, and
what the trained network gains (the learned values themselves are parity
unpinned: any trained weights are valid).

Data: serial F (FP32 increment form) at 129^2 over 64 slices of T = 1 for
seed-drawn instances, restricted to the 64 x 64 operator grid.  The gain is
measured on held-out instances as the one-slice prediction error (data term)
of G = B(tau1) + P_s(w + s * FNO(w)) against F: trained versus untrained
network and versus the propagator without the network (FNO output zero).
"""
import numpy as np
import pytest

from helpers import say
from oracle import fno as ofno
from synthetic import plain_at_scale

pytestmark = pytest.mark.gpu

DT = 1.0 / 64


@pytest.fixture(scope="module")
def data():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_02521_amd.train import generate_pairs
    say("fno training data")
    tr = generate_pairs([plain_at_scale(1000 + i, M=129) for i in range(24)])
    va = generate_pairs([plain_at_scale(2000 + i, M=129) for i in range(4)])
    return tr, va


def test_pairs_are_finite_and_consistent(data):
    """Every pair is finite; V_in = B0 + w_in holds on the ring (w_in = 0 there),
    and V_in, V_tgt carry the Dirichlet ring of their times."""
    import torch
    (pairs, meta), _ = data
    assert pairs.shape == (24 * 64, 4, 64, 64)
    assert bool(torch.isfinite(pairs).all())
    ring = torch.ones(64, 64, dtype=torch.bool, device=pairs.device)
    ring[1:-1, 1:-1] = False
    assert float(pairs[:, 0][:, ring].abs().max()) == 0.0
    # targets change little over one slice compared with their size
    d = (pairs[:, 3] - pairs[:, 2]).abs().max() / pairs[:, 2].abs().max()
    assert 0.0 < float(d) < 0.2


def test_training_gain(data):
    import torch
    from paper_2404_02521_amd import _lib as L
    from paper_2404_02521_amd.fno import Fno
    from paper_2404_02521_amd.train import evaluate, train
    (pairs, meta), (vp, vm) = data
    flat = torch.from_numpy(ofno.flatten(ofno.init_params(np.random.default_rng(0)))
                            .astype(np.float32)).cuda()
    say("fno training gain")
    net = Fno(max_batch=64, out_scale=DT)
    net.set_params(flat)
    untrained = evaluate(net, vp, vm, DT)
    zero = Fno(max_batch=64, out_scale=DT)
    zero.set_params(torch.zeros_like(flat))
    without = evaluate(zero, vp, vm, DT)
    hist = train(net, pairs, meta, DT, epochs=60, batch=64, precision=L.PR_FNO_BF16, lam=1.0,
                 log_every=10)
    trained = evaluate(net, vp, vm, DT)
    print("[gain] data term: untrained %.3e, without network %.3e, trained %.3e (%d steps)"
          % (untrained[1], without[1], trained[1], hist[-1][1]), flush=True)
    assert all(np.isfinite(h[2]) for h in hist)
    assert trained[1] < 0.5 * untrained[1]
    assert trained[1] < 0.9 * without[1]
    net.close()
    zero.close()
