"""The oracle against its frozen record (tests/golden/c1_oracle.txt, written by
tests/golden/make_golden.py from the oracle alone): serial F at sample nodes
and the Parareal iteration history on the 65^2 FP64 configuration."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_oracle.txt")


def _problem(name):
    kind = oracle.PAYOFF_BASKET if name == "basket" else oracle.PAYOFF_EXCHANGE
    return oracle.Problem(M=65, sigma1=0.3, sigma2=0.2, rho=0.5, r=0.05, payoff_kind=kind,
                          w1=0.5, w2=0.5, strike=1.0)


def test_oracle_matches_golden_record():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    cache = {}
    for r in rows:
        name = r[1]
        p = _problem(name)
        if r[0] == "F":
            if name not in cache:
                cache[name] = oracle.serial_fine(p, 8, 1.0, 128)
            assert abs(cache[name][int(r[2]), int(r[3])] - float(r[4])) <= 1e-14
        else:
            _, K, inc = oracle.parareal_bs(p, p.with_M(33), 8, 1.0, 128, 64, tol=1e-8)
            assert K == int(r[2])
            assert np.allclose(inc, [float(x) for x in r[3:]], rtol=1e-12, atol=1e-16)
