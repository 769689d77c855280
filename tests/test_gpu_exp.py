"""Stored-segment (EXP) sweep and work-unit schedules (paper sections 4.2 and
4.3) against the on-the-fly sweep and the FP64 oracle.

The replay kernel reads the pieces that the per-lane walk generated and runs
the same FP32 arithmetic on them in the same order per lane, so after one
iteration from zero flux every outgoing boundary flux must be bit for bit the
on-the-fly one; later iterates differ only through the order of FP64 tally
additions.  The schedules change only which workgroup sweeps
which unit, so they agree to the same level.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_17743_amd import problems as P

pytestmark = pytest.mark.gpu

# Later iterates: the FP64 tallies are summed in a different order, which now
# and then moves an FP32 reduced source by one rounding (1e-7 relative); a
# wrong piece or weight would move the flux by far more than this.
PHI_RTOL = 1e-6


@pytest.fixture(scope="module")
def moc():
    import torch
    assert torch.cuda.is_available()
    from paper_2503_17743_amd import moc as M
    M.lib()
    return M


def _all_slots(plan):
    return np.arange(2 * plan.info["n_3d_tracks"], dtype=np.int64)


def _run(moc, plan, prob, iters, store=None, schedule=None):
    s = moc.Solver(plan, fp64_boundary=False)
    s.set_source(prob.q)
    if schedule is not None:
        s.set_schedule(*schedule)
    info = None
    if store is not None:
        info = s.store_segments(**store)
    s.reset()
    s.iterate(1)
    psi1 = s.boundary_flux(_all_slots(plan))
    st = s.iterate(iters - 1) if iters > 1 else None
    phi = s.flux()
    s.close()
    return phi, psi1, info, st


@pytest.mark.parametrize("name", ["small", "lattice8"])
def test_replay_equals_on_the_fly(moc, name, nthreads):
    prob = P.small_lattice() if name == "small" else P.get(name)
    plan = moc.Plan(prob)
    phi0, psi0, _, _ = _run(moc, plan, prob, 6)
    phi1, psi1, info, st = _run(moc, plan, prob, 6, store=dict(fraction=0.8))
    print(name, info)
    assert info["units_stored"] == info["units_total"]
    assert info["wave_steps_stored"] == info["wave_steps_total"] > 0
    assert st["link_errors"] == 0
    np.testing.assert_array_equal(psi1, psi0)
    np.testing.assert_allclose(phi1, phi0, rtol=PHI_RTOL)
    if name == "small":
        ophi, _ = O.Model(prob, n_threads=nthreads).solve(max_iters=6, tol=0.0)
        assert np.max(np.abs(phi1 - ophi) / ophi) < 1e-5


def test_partial_store_takes_the_largest_units(moc):
    """A store too small for every unit keeps the units of largest footprint;
    the rest run on the fly in the same iteration."""
    prob = P.get("lattice8")
    plan = moc.Plan(prob)
    phi0, psi0, _, _ = _run(moc, plan, prob, 4)
    # count first to learn the full footprint, then give a third of it
    s = moc.Solver(plan, fp64_boundary=False)
    full = s.store_segments(fraction=0.8)["bytes_all"]
    s.close()
    phi1, psi1, info, _ = _run(moc, plan, prob, 4, store=dict(fraction=0.8, max_bytes=full // 3))
    print(info)
    assert 0 < info["units_stored"] < info["units_total"]
    assert info["bytes_used"] <= full // 3
    # the largest units hold a larger share of the steps than of the units
    assert (info["wave_steps_stored"] / info["wave_steps_total"]
            > info["units_stored"] / info["units_total"])
    np.testing.assert_array_equal(psi1, psi0)
    np.testing.assert_allclose(phi1, phi0, rtol=PHI_RTOL)


@pytest.mark.parametrize("order,persistent", [("natural", False), ("alternating", False),
                                              ("natural", True), ("longest_first", True),
                                              ("alternating", True)])
def test_schedules_agree(moc, order, persistent):
    prob = P.get("lattice8")
    plan = moc.Plan(prob)
    phi0, psi0, _, _ = _run(moc, plan, prob, 4)
    phi1, psi1, _, _ = _run(moc, plan, prob, 4, schedule=(order, persistent))
    np.testing.assert_array_equal(psi1, psi0)
    np.testing.assert_allclose(phi1, phi0, rtol=PHI_RTOL)
    # and with the store replayed under the same schedule
    phi2, psi2, _, _ = _run(moc, plan, prob, 4, schedule=(order, persistent),
                            store=dict(fraction=0.8))
    np.testing.assert_array_equal(psi2, psi0)
    np.testing.assert_allclose(phi2, phi0, rtol=PHI_RTOL)


def test_store_rejects_other_sweeps(moc):
    """The store records the per-lane FP32 walk: a problem with more than 8
    groups (groups split across lanes) is rejected."""
    prob = P.small_lattice(n_groups=12)
    plan = moc.Plan(prob)
    s = moc.Solver(plan)
    with pytest.raises(moc.MocError) as e:
        s.store_segments(fraction=0.5)
    assert e.value.code == moc.MOC_EINVAL
    s.close()


@pytest.mark.parametrize("name,sizes", [("small", (256, 512, 1024)), ("lattice8", (256, 512, 1024)),
                                        ("lattice32", (512, 1024))])
def test_window_sizes_agree(moc, name, sizes):
    """Windows end at 2D segment boundaries and the walk evaluates every plane
    crossing from its index, so the pieces of a line do not depend on the
    window length: the outgoing boundary flux after one iteration is the
    same bit for bit for every workgroup size, and the flux agrees up to the
    order of FP64 tally additions."""
    import torch
    prob = P.small_lattice() if name == "small" else P.get(name)
    plan = moc.Plan(prob)
    rng = np.random.default_rng(5)
    n_slots = 2 * plan.info["n_3d_tracks"]
    slots = np.sort(rng.choice(n_slots, size=min(n_slots, 1_000_000), replace=False))
    ref = None
    for nt in sizes:
        s = moc.Solver(plan, fp64_boundary=False)
        s.set_window(nt)
        assert s.window()[0] == nt
        s.set_source(prob.q)
        s.iterate(1)
        psi = s.boundary_flux(slots)
        s.iterate(2)
        phi = s.flux()
        s.close()
        del s
        torch.cuda.empty_cache()
        if ref is None:
            ref = (psi, phi)
        else:
            np.testing.assert_array_equal(psi, ref[0])
            np.testing.assert_allclose(phi, ref[1], rtol=PHI_RTOL)


@pytest.mark.parametrize("name,threads", [("small", 256), ("lattice8", 256), ("lattice8", 1024),
                                          ("lattice32", 1024)])
def test_bundle_assignment_agrees(moc, name, threads):
    """Static and dynamic assignment of a window's bundles to the waves change
    only which wave sweeps a line: the outgoing boundary flux after one
    iteration is the same bit for bit, and the flux agrees up to the order of
    FP64 tally additions.  The stored-segment replay indexes its pieces by
    bundle, so it agrees under either assignment too."""
    prob = P.small_lattice() if name == "small" else P.get(name)
    plan = moc.Plan(prob)
    rng = np.random.default_rng(7)
    n_slots = 2 * plan.info["n_3d_tracks"]
    slots = np.sort(rng.choice(n_slots, size=min(n_slots, 1_000_000), replace=False))
    ref = None
    for mode, store in (("static", False), ("dynamic", False), ("dynamic", True), ("static", True)):
        if store and name == "lattice32":
            continue
        s = moc.Solver(plan, fp64_boundary=False)
        s.set_window(threads)
        s.set_bundles(mode)
        s.set_source(prob.q)
        if store:
            info = s.store_segments(fraction=0.8)
            assert info["units_stored"] == info["units_total"]
            s.reset()
        s.iterate(1)
        psi = s.boundary_flux(slots)
        st = s.iterate(2)
        phi = s.flux()
        s.close()
        del s
        assert st["link_errors"] == 0
        if ref is None:
            ref = (psi, phi)
        else:
            np.testing.assert_array_equal(psi, ref[0])
            np.testing.assert_allclose(phi, ref[1], rtol=PHI_RTOL)
