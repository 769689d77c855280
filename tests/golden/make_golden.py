"""Writes the stored expected values under tests/golden/ from the FP64 oracle
only (no HIP code is imported).  Run from the repository root:

    python tests/golden/make_golden.py

small_lattice_5it.txt: the flux after 5 Jacobi source iterations (Eqs. 3-4,
phi^0 = 0, vacuum and reflective boundaries as in the problem) of the seeded
3x3 small lattice, one line per FSR with its G group fluxes.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O                      # noqa: E402
from paper_2503_17743_amd import problems as P      # noqa: E402


def main():
    prob = P.small_lattice()
    phi, res = O.Model(prob, n_threads=8).solve(max_iters=5, tol=0.0)
    path = os.path.join(HERE, "small_lattice_5it.txt")
    with open(path, "w") as f:
        f.write("# FP64 oracle: 5 source iterations of problems.small_lattice() (seed 11)\n")
        f.write(f"# n_fsr {phi.shape[0]} groups {phi.shape[1]}; leakage {res['leakage']:.17g}\n")
        np.savetxt(f, phi, fmt="%.17g")
    print("wrote", path)


if __name__ == "__main__":
    main()
