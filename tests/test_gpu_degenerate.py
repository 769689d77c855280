"""Degenerate and boundary inputs on the GPU, against the FP64 oracle: a
zero source, one axial layer, the smallest quadrature in an all-vacuum pure
absorber, and a source confined to one FSR."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_17743_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def moc():
    import torch
    assert torch.cuda.is_available()
    from paper_2503_17743_amd import moc as M
    M.lib()
    return M


def _run(moc, p, iters, fp64=False):
    s = moc.Solver(moc.Plan(p))
    s.set_source(p.q)
    st = s.iterate(iters, sweep_fp64=fp64)
    return s.flux(), st


def _rel(a, b):
    m = np.abs(b) > 0
    return float(np.max(np.abs(a[m] - b[m]) / np.abs(b[m]))) if m.any() else 0.0


def test_zero_source_gives_zero_flux(moc):
    p = P.small_lattice()
    p.q = np.zeros_like(p.q)
    s = moc.Solver(moc.Plan(p))
    s.set_source(p.q)
    phi, st = s.solve(tol=1e-6, max_iters=50)
    assert st["converged"] and st["iters"] == 2
    assert (phi == 0).all()
    assert st["leakage"] == 0 and st["balance_lhs"] == 0


@pytest.mark.parametrize("fp64", [False, True])
def test_single_axial_layer(moc, nthreads, fp64):
    p = P.small_lattice(seed=31, n_layers=1, height=1.0)
    phi, st = _run(moc, p, 4, fp64)
    ophi, _ = O.Model(p, n_threads=nthreads).solve(max_iters=4, tol=0.0)
    assert _rel(phi, ophi) < (1e-10 if fp64 else 1e-5)
    assert st["link_errors"] == 0


@pytest.mark.parametrize("fp64", [False, True])
def test_minimal_quadrature_vacuum_absorber(moc, nthreads, fp64):
    """4 azimuthal x 2 polar angles, vacuum on every face, no scattering: one
    iteration is the exact answer (the source does not depend on the flux)."""
    p = P.pure_absorber(n_groups=2, q=[1.0, 0.5], n_azim=4, n_polar=2)
    phi, st = _run(moc, p, 2, fp64)
    ophi, ores = O.Model(p, n_threads=nthreads).solve(max_iters=2, tol=0.0)
    assert _rel(phi, ophi) < (1e-10 if fp64 else 1e-5)
    assert ores["residual"] < 1e-12        # already converged after one iteration
    # absorption + leakage = source for a pure absorber
    assert abs(st["absorption"] + st["leakage"] - st["source"]) < (1e-9 if fp64 else 1e-5) * st["source"]


@pytest.mark.parametrize("fp64", [False, True])
def test_source_in_one_fsr(moc, nthreads, fp64):
    """A point-like source (one FSR, one group): the flux elsewhere comes only
    from transport and scattering, including FSRs many orders below the peak."""
    p = P.small_lattice(seed=33)
    p.q = np.zeros_like(p.q)
    p.q[p.n_fsr // 2, 0] = 1.0
    phi, st = _run(moc, p, 5, fp64)
    ophi, _ = O.Model(p, n_threads=nthreads).solve(max_iters=5, tol=0.0)
    assert ((phi > 0) == (ophi > 0)).all()
    assert _rel(phi, ophi) < (1e-10 if fp64 else 1e-5)
