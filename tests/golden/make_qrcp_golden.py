"""Writes tests/golden/qrcp_2560x2048_sep105.txt: the oracle's QR with column
pivoting of a 2560 x 2048 sketch-shaped matrix (the sketch shape of the
4,194,304 x 2,048 workload, d = ceil(1.25 n) = 2560), which the oracle needs
about two minutes to factor, too long to run inside the GPU test.

Input: ``workloads.column_scaled_well_separated(2560, 2048, seed=2560*7+2048,
ratio=1.05)`` (Gaussian columns scaled 1.05^-rank apart, so every pivot
decision has a margin; LAPACK's GEQP3 through scipy picks the same pivots).
Stored: the 0-based pivot order J, the diagonal of R and its first
superdiagonal (R = the oracle's upper-triangular factor, non-negative
diagonal). Only ``oracle/`` computes them.

Run from the repository root:  python tests/golden/make_qrcp_golden.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cqrrpt_oracle as O  # noqa: E402
from paper_2311_08316_amd import workloads as W  # noqa: E402

D, N, RATIO = 2560, 2048, 1.05
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "qrcp_2560x2048_sep105.txt")


def main():
    X = W.column_scaled_well_separated(D, N, seed=D * 7 + N, ratio=RATIO)
    J, R = O.qrcp(X)
    with open(OUT, "w") as fh:
        fh.write("# Oracle QRCP (Householder, max-norm pivoting, exact norm recompute) of\n")
        fh.write(f"# workloads.column_scaled_well_separated({D}, {N}, seed={D * 7 + N}, "
                 f"ratio={RATIO}).\n")
        fh.write("# Written by tests/golden/make_qrcp_golden.py (calls only oracle/).\n")
        fh.write("# Columns: i, J[i], R[i,i], R[i,i+1] (0 past the last column), "
                 "values as float.hex.\n")
        for i in range(N):
            sup = R[i, i + 1] if i + 1 < N else 0.0
            fh.write(f"{i} {int(J[i])} {float(R[i, i]).hex()} {float(sup).hex()}\n")
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
