"""Write tests/golden/c1_oracle.txt from the FP64 oracle (calls only oracle/).

The 65 x 65 FP64 configuration (sigma1 0.3, sigma2 0.2, rho 0.5, r 0.05, T 1,
N = 8 slices, F 128 steps per slice, G 33 x 33 at 64 steps per slice,
absolute tolerance 1e-8): serial F at a few nodes and the Parareal iteration
history (Eq. (parareal), Sec. 3.1) for the basket call (0.5, 0.5, K = 1) and
the exchange option.  A frozen record of the oracle: a later change to its
arithmetic shows up against it.  Run from the repository root:

    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402

NODES = [(8, 8), (16, 16), (16, 32), (32, 16), (32, 32), (48, 48)]   # S = 0.0625 * index


def main():
    lines = ["# FP64 oracle on the 65^2 configuration; written by tests/golden/make_golden.py",
             "# payoff node_i node_j serial_F   |  payoff K increments..."]
    for name, kind in (("basket", oracle.PAYOFF_BASKET), ("exchange", oracle.PAYOFF_EXCHANGE)):
        p = oracle.Problem(M=65, sigma1=0.3, sigma2=0.2, rho=0.5, r=0.05, payoff_kind=kind,
                           w1=0.5, w2=0.5, strike=1.0)
        pc = p.with_M(33)
        u = oracle.serial_fine(p, 8, 1.0, 128)
        for i, j in NODES:
            lines.append("F %s %d %d %.17g" % (name, i, j, u[i, j]))
        _, K, inc = oracle.parareal_bs(p, pc, 8, 1.0, 128, 64, tol=1e-8)
        lines.append("P %s %d %s" % (name, K, " ".join("%.17g" % x for x in inc)))
    with open(os.path.join(HERE, "c1_oracle.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
