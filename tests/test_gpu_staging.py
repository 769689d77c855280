"""Window staging of the FP32 sweep against the FP64 oracle on its less common
paths: windows of more than 64 2D segments (each reduced-source entry's region
read from HBM instead of from the lane that holds it) with rows of a multiple
of four FSR-groups (16-byte direct gathers into LDS) and without (4-byte)."""
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


@pytest.mark.parametrize("groups", [4, 3])
def test_windows_of_more_than_64_segments(moc, nthreads, groups):
    # 12x12 cells of 8 sectors x 2 rings, one layer: 2D tracks of up to 80
    # segments, each swept in one window (K x G = 4 or 3 entries per segment)
    p = P.small_lattice(seed=41, n=12, height=1.0, n_layers=1, n_groups=groups, n_sectors=8,
                        radius=0.4, n_azim=8, n_polar=2)
    plan = moc.Plan(p)
    _, _, first = plan.segments2d()
    assert np.diff(first).max() > 64
    s = moc.Solver(plan, fp64_boundary=False)
    assert s.window()[1] > 64
    s.set_source(p.q)
    st = s.iterate(4)
    phi = s.flux()
    s.close()
    ophi, _ = O.Model(p, n_threads=nthreads).solve(max_iters=4, tol=0.0)
    m = ophi > 0
    assert ((phi > 0) == m).all()
    assert np.max(np.abs(phi[m] - ophi[m]) / ophi[m]) < 1e-5
    assert st["link_errors"] == 0
