"""Continuous-batching server on the GPU: every result is the same alone and
in the mix, matches the FP64 oracle, and admission respects the arena."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_17743_amd import problems as P

pytestmark = pytest.mark.gpu

TOL = 1e-6
MAX_IT = 400


@pytest.fixture(scope="module")
def moc():
    import torch
    assert torch.cuda.is_available()
    from paper_2503_17743_amd import moc as M
    M.lib()
    return M


def _mix():
    # varied sizes, group counts, layers and quadratures in one batch
    return [
        P.small_lattice(seed=21, n=2, n_groups=1, n_layers=2, height=2.0, n_azim=8, n_polar=2),
        P.small_lattice(seed=22, n=3, n_groups=3, n_layers=3, height=3.0, n_azim=8, n_polar=4),
        P.small_lattice(seed=23, n=4, n_groups=7, n_layers=4, height=4.0, n_azim=12, n_polar=6,
                        radial=0.15, axial=0.25),
        P.small_lattice(seed=24, n=2, n_groups=5, n_layers=6, height=6.0, n_azim=16, n_polar=2,
                        radial=0.1, axial=0.3, n_sectors=8, radius=0.4),
        P.small_lattice(seed=25, n=3, n_groups=2, n_layers=2, height=2.0, n_azim=4, n_polar=4,
                        bc=(1, 1, 1, 1, 1, 1)),
        P.small_lattice(seed=26, n=5, n_groups=4, n_layers=3, height=1.5, n_azim=8, n_polar=4,
                        radial=0.2, axial=0.2),
    ]


def _alone(moc, prob):
    s = moc.Solver(moc.Plan(prob), fp64_boundary=False)
    s.set_source(prob.q)
    return s.solve(tol=TOL, max_iters=MAX_IT)


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def _serve(moc, probs, arena_bytes, max_slots=64, fill_units=None):
    srv = moc.Server(arena_bytes, max_slots=max_slots, fill_units=fill_units)
    plans = [moc.Plan(p) for p in probs]
    tickets = [srv.submit(pl, p.q, TOL, MAX_IT) for pl, p in zip(plans, probs)]
    results = {}
    max_active = 0
    steps = 0
    while len(results) < len(tickets):
        na, nq = srv.step()
        steps += 1
        assert steps < 100000
        for i, tk in enumerate(tickets):
            if i in results:
                continue
            r = srv.poll(tk)
            if r is not None:
                results[i] = r
        max_active = max(max_active, na)
    srv.close()
    return [results[i] for i in range(len(probs))], max_active, plans


def test_alone_equals_mix(moc):
    probs = _mix()
    mixed, max_active, plans = _serve(moc, probs, arena_bytes=2 << 30)
    assert max_active >= 2
    for p, (phi_m, st_m) in zip(probs, mixed):
        phi_a, st_a = _alone(moc, p)
        assert st_m["converged"] and st_a["converged"]
        # the device applies moc_solve's stopping rule to each request, so a
        # served request stops at the same iteration as a plain solve (its
        # residual would have to fall within FP rounding of tol to differ)
        assert st_m["iters"] == st_a["iters"], (st_m["iters"], st_a["iters"])
        assert _rel(phi_m, phi_a) < 1e-5, p.name
        assert st_m["link_errors"] == 0


def test_served_results_match_oracle(moc, nthreads):
    probs = _mix()[1:3]
    mixed, _, _ = _serve(moc, probs, arena_bytes=1 << 30)
    for p, (phi, st) in zip(probs, mixed):
        ophi, _ = O.Model(p, n_threads=nthreads).solve(tol=1e-12, max_iters=2000)
        assert _rel(phi, ophi) < 1e-5, p.name


def test_admission_by_footprint(moc):
    """An arena that holds only about two requests at a time: requests wait,
    are admitted as others retire, and all finish with the same results."""
    probs = [P.small_lattice(seed=30 + i, n=3, n_groups=3, n_layers=3, height=3.0) for i in range(5)]
    need = max(moc.Plan(p).info["workspace_bytes"] for p in probs)
    tables = moc.Server.overhead_bytes(64)     # server tables at the front of the arena
    mixed, max_active, _ = _serve(moc, probs, arena_bytes=tables + int(2.5 * need))
    assert 1 <= max_active <= 2
    for p, (phi, st) in zip(probs, mixed):
        phi_a, _ = _alone(moc, p)
        assert _rel(phi, phi_a) < 1e-5


def test_slot_limit(moc):
    probs = [P.small_lattice(seed=40 + i, n=2, n_groups=2, n_layers=2, height=2.0) for i in range(4)]
    mixed, max_active, _ = _serve(moc, probs, arena_bytes=1 << 30, max_slots=1)
    assert max_active == 1
    for p, (phi, st) in zip(probs, mixed):
        phi_a, _ = _alone(moc, p)
        assert _rel(phi, phi_a) < 1e-5


def test_fill_target_admission(moc):
    """With a fill target below one request's work, requests run one at a
    time in arrival order; with a large one they all share the GPU."""
    probs = [P.small_lattice(seed=60 + i, n=2, n_groups=2, n_layers=2, height=2.0) for i in range(4)]
    one, max_one, _ = _serve(moc, probs, arena_bytes=1 << 30, fill_units=1)
    assert max_one == 1
    many, max_many, _ = _serve(moc, probs, arena_bytes=1 << 30, fill_units=0)
    assert max_many == len(probs)
    for (phi_a, _), (phi_b, _) in zip(one, many):
        assert _rel(phi_a, phi_b) < 1e-12


def test_two_class_driver_matches_one_server(moc):
    """The serving driver with two servers (small requests on their own
    stream) gives every request the same result and iteration count as one
    server, under Poisson arrivals."""
    from paper_2503_17743_amd import serve as S
    probs = _mix()
    reqs = P.with_arrivals(probs, 200.0, seed=9)
    plans = [moc.Plan(p) for p in probs]
    arena = moc.Server.overhead_bytes(64) + (1 << 30)
    phi1, d1 = S.run_stream(reqs, plans, TOL, MAX_IT, arena, use_arrivals=True)
    # split so that both servers get requests
    units = sorted(2 * pl.info["n_2d_tracks"] for pl in plans)
    split = units[len(units) // 2]
    phi2, d2 = S.run_stream(reqs, plans, TOL, MAX_IT, arena, use_arrivals=True, classes=2,
                            split_units=split)
    # the same arithmetic per request; only the order of FP64 tally additions
    # differs (and through it, rarely, one FP32 rounding of the reduced source)
    for a, b, s1, s2 in zip(phi1, phi2, d1["stats"], d2["stats"]):
        assert s1["iters"] == s2["iters"]
        assert _rel(b, a) < 1e-6


def test_server_rejects_invalid(moc):
    import ctypes as C
    srv = moc.Server(moc.Server.overhead_bytes(4) + (64 << 20), max_slots=4)
    p = P.small_lattice(seed=50, n=2, n_groups=2, n_layers=2, height=2.0)
    pl = moc.Plan(p)
    q = np.ascontiguousarray(p.q)
    t = C.c_ulonglong()
    bad = moc.SolveOpts(1e-6, 100, 1, 0)          # FP64 sweep is not served
    assert moc.lib().moc_server_submit(srv._h, pl._h, q.ctypes.data_as(C.c_void_p), C.byref(bad),
                                       C.byref(t)) == moc.MOC_EINVAL
    st = moc.Stats()
    assert moc.lib().moc_server_poll(srv._h, C.c_ulonglong(12345), C.byref(st), None, 0) == moc.MOC_EINVAL
    big = P.config_lattice8()
    with pytest.raises(moc.MocError) as e:
        srv.submit(moc.Plan(big), big.q)
    assert e.value.code == moc.MOC_ENOMEM
    srv.close()
