"""Writes the stored expected values under tests/golden from the CPU oracle only.

Run from the repository root:  python tests/golden/make_golden.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def main():
    # Mode counts of a 64^3 mesh, unit-k_f bins from 0 to the Nyquist index
    # (FFTPower binning, Sec. 3.4.1; integer n^2 rule, DC excluded).
    tab = oracle.mode_tables(64, 1000.0, 0.0, 1.0, 32)
    np.savetxt(os.path.join(HERE, "modecounts_n64_dk1.txt"), tab["modes"], fmt="%d",
               header="64^3 mesh, k-bins [b, b+1) k_f, b = 0..31: Hermitian-weighted "
                      "mode counts (oracle.mode_tables)")
    tab = oracle.mode_tables(64, 1000.0, 0.0, 1.0, 32, nmu=5)
    np.savetxt(os.path.join(HERE, "modecounts2d_n64_dk1_nmu5.txt"), tab["modes2d"],
               fmt="%d", header="64^3 mesh, 32 k-bins x 5 |mu| bins, line of sight z")


if __name__ == "__main__":
    main()
