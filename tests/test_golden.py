"""Stored oracle values (tests/golden/, written by tests/golden/make_golden.py
from the oracle only): the oracle reproduces them (CPU), and the HIP path
matches them to the FP32 bar (GPU)."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_17743_amd import problems as P

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "small_lattice_5it.txt")


def _golden():
    return np.loadtxt(GOLDEN, comments="#")


def test_oracle_reproduces_golden(nthreads):
    phi, _ = O.Model(P.small_lattice(), n_threads=nthreads).solve(max_iters=5, tol=0.0)
    np.testing.assert_allclose(phi, _golden(), rtol=1e-12, atol=0)


@pytest.mark.gpu
def test_hip_path_matches_golden():
    import torch
    assert torch.cuda.is_available()
    from paper_2503_17743_amd import moc
    prob = P.small_lattice()
    s = moc.Solver(moc.Plan(prob))
    s.set_source(prob.q)
    s.iterate(5)
    g = _golden()
    assert np.max(np.abs(s.flux() - g) / g) < 1e-5
