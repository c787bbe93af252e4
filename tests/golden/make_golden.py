"""Writes oracle_random_n12_seed7.txt: a regression fixture produced by the
oracle alone (random skew matrix of order 12, seed 7, all 6 non-negative
eigenvalues).  Run from the repository root: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1912_04062_amd import workloads  # noqa: E402


def main():
    A = workloads.random_skew(12, 7)
    lam, _ = oracle.skew_evd(A)
    path = os.path.join(HERE, "oracle_random_n12_seed7.txt")
    with open(path, "w") as f:
        f.write("# written by tests/golden/make_golden.py (oracle only):\n")
        f.write("# eigenvalue magnitudes of workloads.random_skew(12, 7), ascending\n")
        f.write(" ".join(f"{x:.17e}" for x in lam) + "\n")


if __name__ == "__main__":
    main()
