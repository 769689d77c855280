"""Group counts above 8: groups split into chunks of at most 8 across lanes
(T = 64 / chunks lines per wave), up to the maximum of 64 groups.  Fixed
source iterations against the FP64 oracle with the FP32 and FP64 sweeps, and
the batched serving sweep with such a problem in the mix."""
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


def _rel(a, b):
    m = np.abs(b) > 0
    return float(np.max(np.abs(a[m] - b[m]) / np.abs(b[m])))


@pytest.mark.parametrize("G", [9, 12, 24, 64])
@pytest.mark.parametrize("fp64", [False, True])
def test_many_groups_fixed_iterations_match_oracle(moc, nthreads, G, fp64):
    p = P.small_lattice(seed=40 + G, n=2, height=2.0, n_layers=2, n_groups=G, n_azim=8, n_polar=2,
                        radial=0.25, axial=0.4)
    plan = moc.Plan(p)
    chunks = -(-G // 8)
    assert plan.info["tracks_per_wave"] == 64 // chunks
    s = moc.Solver(plan)
    s.set_source(p.q)
    om = O.Model(p, n_threads=nthreads)
    for it in (1, 3):
        s.reset()
        st = s.iterate(it, sweep_fp64=fp64)
        ophi, ores = om.solve(max_iters=it, tol=0.0)
        err = _rel(s.flux(), ophi)
        print(f"G={G} fp64={fp64} {it} iterations: max rel err {err:.3e}")
        assert err < (1e-10 if fp64 else 1e-5), err
        assert st["link_errors"] == 0
        assert st["seg_group_updates"] == 2 * om.info["n_segments"] * G


def test_many_groups_served_in_a_mix(moc):
    """A 12-group request (chunked lanes) beside one-chunk requests in the
    batched sweep: each result as a plain solve gives it."""
    probs = [P.small_lattice(seed=71, n=2, height=2.0, n_layers=2, n_groups=12, n_azim=8, n_polar=2,
                             radial=0.25, axial=0.4),
             P.small_lattice(seed=72, n=3, n_groups=3),
             P.small_lattice(seed=73, n=2, n_groups=7, n_layers=4, height=4.0)]
    srv = moc.Server(moc.Server.overhead_bytes(64) + (1 << 30), fill_units=0)
    plans = [moc.Plan(p) for p in probs]
    tickets = [srv.submit(pl, p.q, 1e-6, 400) for pl, p in zip(plans, probs)]
    out, steps, max_active = {}, 0, 0
    while len(out) < len(tickets):
        na, _ = srv.step()
        max_active = max(max_active, na)
        steps += 1
        assert steps < 10000
        for i, tk in enumerate(tickets):
            if i not in out:
                r = srv.poll(tk)
                if r is not None:
                    out[i] = r
    srv.close()
    assert max_active == len(probs)
    for i, (p, pl) in enumerate(zip(probs, plans)):
        s = moc.Solver(pl, fp64_boundary=False)
        s.set_source(p.q)
        phi_a, st_a = s.solve(tol=1e-6, max_iters=400)
        phi_m, st_m = out[i]
        assert st_m["converged"] and st_a["converged"]
        assert st_m["iters"] == st_a["iters"]
        assert _rel(phi_m, phi_a) < 1e-5


@pytest.mark.parametrize("fp64", [False, True])
def test_direct_sweep_when_the_window_does_not_fit(moc, nthreads, fp64):
    """160 layers x 48 groups: one 2D segment's reduced source and FP64 tally
    (160 * 48 * 12 B = 92 KB) exceed the LDS window budget, so the sweep takes
    the direct path (one wave per bundle, FP64 atomics per piece)."""
    p = P.small_lattice(seed=50, n=2, height=40.0, n_layers=160, n_groups=48, n_azim=4, n_polar=2,
                        radial=0.3, axial=0.5)
    assert p.n_layers * p.n_groups * 12 > 78 * 1024
    plan = moc.Plan(p)
    s = moc.Solver(plan)
    s.set_source(p.q)
    om = O.Model(p, n_threads=nthreads)
    st = s.iterate(2, sweep_fp64=fp64)
    ophi, _ = om.solve(max_iters=2, tol=0.0)
    err = _rel(s.flux(), ophi)
    print(f"direct sweep fp64={fp64}: max rel err {err:.3e}")
    assert err < (1e-10 if fp64 else 1e-5)
    assert st["link_errors"] == 0
    assert st["seg_group_updates"] == 2 * om.info["n_segments"] * p.n_groups
