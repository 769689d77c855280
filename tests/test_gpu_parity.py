"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances.  The oracle and the planner share the laydown definition, so
every FSR id and segment count must agree exactly and lengths to FP64
rounding.  The FP32 sweep keeps angular flux and segment arithmetic in FP32
(unit roundoff 6e-8, stable 1-e^-tau within 2 ulp) with FP64 tallies; the
bar for fluxes is the 1e-5 max relative FSR error.  The FP64 sweep mode is
held to 1e-10 (rounding and atomic order only).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_17743_amd import problems as P

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-10


@pytest.fixture(scope="module")
def moc():
    import torch
    assert torch.cuda.is_available()
    from paper_2503_17743_amd import moc as M
    M.lib()
    return M


def _solver(moc, prob):
    plan = moc.Plan(prob)
    s = moc.Solver(plan)
    s.set_source(prob.q)
    return plan, s


def _relerr(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def test_plain_box_closed_form(moc, nthreads):
    """FP64 plain method to residual 1e-10: phi = Q/(St - Ss) = 2 in all FSRs."""
    prob = P.config_plain()
    plan, s = _solver(moc, prob)
    phi, st = s.solve(tol=1e-10, max_iters=2000, sweep_fp64=True)
    assert st["converged"] and st["link_errors"] == 0
    np.testing.assert_allclose(phi, 2.0, rtol=1e-9)
    om = O.Model(prob, n_threads=nthreads)
    ophi, ores = om.solve()
    assert _relerr(phi, ophi) < TOL64
    # the FP32 sweep reaches the same value to its own precision
    phi32, st32 = s.solve(tol=1e-7, max_iters=2000)
    assert _relerr(phi32, ophi) < TOL32


def test_volumes_and_counts_match_oracle(moc, nthreads):
    prob = P.small_lattice()
    plan, s = _solver(moc, prob)
    om = O.Model(prob, n_threads=nthreads)
    np.testing.assert_allclose(s.volumes(), om.volumes(), rtol=1e-12)
    st = s.iterate(1)
    assert st["seg_group_updates"] == 2 * om.info["n_segments"] * prob.n_groups
    assert st["link_errors"] == 0


TRACE_CASES = [
    # 45-degree azimuths on square lattices: tracks along sector lines and
    # through cell centres and corners
    dict(seed=3, n=4, n_azim=12, n_polar=6, radial=0.13, axial=0.17, height=2.3, n_layers=5,
         n_sectors=16),
    dict(seed=9, n=4, n_azim=20, n_polar=4, radial=0.1, axial=0.2, height=4.0, n_layers=4,
         n_sectors=8, radius=0.4),
    dict(seed=10, n=2, n_azim=28, n_polar=2, radial=0.07, axial=0.11, height=1.0, n_layers=3,
         n_sectors=2, radius=0.3, bc=(1, 1, 1, 1, 1, 1)),
]


@pytest.mark.parametrize("case", range(len(TRACE_CASES)))
def test_traced_segments_match_oracle(moc, nthreads, case):
    """OTF generation on the GPU (2D segments + axial splitting) vs brute-force
    3D ray tracing: identical FSR sequences, lengths to FP64 rounding."""
    prob = P.small_lattice(**TRACE_CASES[case])
    plan, s = _solver(moc, prob)
    om = O.Model(prob, trace=False)
    rng = np.random.default_rng(1)
    ids = rng.choice(plan.info["n_3d_tracks"], size=500, replace=False)
    got = s.trace_tracks(ids)
    for tr, (f, l, n) in zip(ids, got):
        fo, lo = om.trace(tr)
        assert n == len(fo), tr
        np.testing.assert_array_equal(f, fo)
        np.testing.assert_allclose(l, lo, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("fp64", [False, True])
def test_small_lattice_fixed_iterations(moc, nthreads, fp64):
    prob = P.small_lattice()
    plan, s = _solver(moc, prob)
    om = O.Model(prob, n_threads=nthreads)
    for iters in (1, 2, 5, 12):
        s.reset()
        st = s.iterate(iters, sweep_fp64=fp64)
        ophi, ores = om.solve(max_iters=iters, tol=0.0)
        err = _relerr(s.flux(), ophi)
        assert err < (TOL64 if fp64 else TOL32), (iters, err)
        assert st["link_errors"] == 0
        assert abs(st["leakage"] - ores["leakage"]) <= (1e-9 if fp64 else 1e-5) * abs(ores["leakage"]) + 1e-30


@pytest.mark.parametrize("fp64", [False, True])
def test_deep_stacks_strided_bundles(moc, nthreads, fp64):
    """A tall, thin lattice (600 lines per stack at any 2D position, 10 per
    layer) where the sweep's bundles take every S-th line (S up to 10) in
    several blocks; fixed iterations against the oracle."""
    prob = P.small_lattice(seed=12, n=2, height=60.0, n_layers=60, n_groups=2, n_azim=4,
                           n_polar=2, axial=0.1)
    plan, s = _solver(moc, prob)
    assert plan.info["line_stride"] == 10
    om = O.Model(prob, n_threads=nthreads)
    for iters in (1, 4):
        s.reset()
        st = s.iterate(iters, sweep_fp64=fp64)
        ophi, ores = om.solve(max_iters=iters, tol=0.0)
        err = _relerr(s.flux(), ophi)
        assert err < (TOL64 if fp64 else TOL32), (iters, err)
        assert st["link_errors"] == 0


@pytest.mark.parametrize("fp64", [False, True])
def test_small_lattice_converged(moc, nthreads, fp64):
    prob = P.small_lattice()
    plan, s = _solver(moc, prob)
    om = O.Model(prob, n_threads=nthreads)
    ophi, ores = om.solve(tol=1e-12)
    phi, st = s.solve(tol=1e-11 if fp64 else 1e-6, max_iters=500, sweep_fp64=fp64)
    assert st["converged"]
    assert _relerr(phi, ophi) < (1e-9 if fp64 else TOL32)
    # particle balance at convergence: absorption + leakage = source
    assert abs(st["absorption"] + st["leakage"] - st["source"]) < 1e-6 * st["source"]
    # per-iteration discrete balance: sum of tallies = psi in - psi out
    assert abs(st["balance_lhs"] - st["balance_rhs"]) < 1e-6 * abs(st["source"])


def test_lattice8_fixed_iterations(moc, nthreads):
    """The 8x8 heterogeneous lattice at full size: 6 source iterations from
    zero, every FSR-group flux within 1e-5 of the FP64 oracle."""
    prob = P.config_lattice8()
    plan, s = _solver(moc, prob)
    om = O.Model(prob, n_threads=nthreads)
    iters = 6
    st = s.iterate(iters)
    ophi, ores = om.solve(max_iters=iters, tol=0.0)
    assert st["seg_group_updates"] == 2 * om.info["n_segments"] * prob.n_groups
    assert st["link_errors"] == 0
    err = _relerr(s.flux(), ophi)
    print(f"lattice8 {iters} iterations: max rel err {err:.3e}")
    assert err < TOL32


@pytest.mark.parametrize("fp64", [False, True])
def test_sweep_items_match_oracle(moc, nthreads, fp64):
    """Sampled single sweep: random bundles, random incoming flux and reduced
    source; tallies and outgoing flux of exactly those tracks."""
    prob = P.config_lattice8()
    plan, s = _solver(moc, prob)
    om = O.Model(prob, trace=False)
    rng = np.random.default_rng(7)
    T, G = plan.info["tracks_per_wave"], prob.n_groups
    items = rng.choice(2 * plan.info["n_chunks"], size=300, replace=False)
    qhat = P.f32(rng.uniform(0.0, 0.2, size=(plan.info["n_fsr"], G)))
    psi_in = P.f32(rng.uniform(0.0, 0.5, size=(len(items), T, G)))
    acc, psi_out = s.sweep_items(items, qhat, psi_in, sweep_fp64=fp64)
    tracks, dirs, rows = [], [], []
    for i, it in enumerate(items):
        ft, nt = plan.chunk(it // 2)
        for k in range(nt):
            tracks.append(ft + k)
            dirs.append(it % 2)
            rows.append((i, k))
    pin = np.array([psi_in[i, k] for i, k in rows])
    oacc, opsi, _ = om.sweep_sample(tracks, dirs, qhat, pin)
    gpsi = np.array([psi_out[i, k] for i, k in rows])
    tol = 1e-12 if fp64 else 2e-6
    np.testing.assert_allclose(gpsi, opsi, rtol=tol, atol=tol * np.abs(opsi).max())
    nz = np.abs(oacc) > 0
    assert (np.abs(acc[~nz]) == 0).all()
    scale = np.abs(oacc).max()
    np.testing.assert_allclose(acc, oacc, rtol=0, atol=(1e-12 if fp64 else 1e-5) * scale)


def test_rerun_is_reproducible(moc):
    prob = P.small_lattice()
    plan, s = _solver(moc, prob)
    s.iterate(10)
    a = s.flux()
    s.reset()
    s.iterate(10)
    b = s.flux()
    assert _relerr(a, b) < 1e-6
    s.reset()
    s.iterate(10, sweep_fp64=True)
    c = s.flux()
    s.reset()
    s.iterate(10, sweep_fp64=True)
    d = s.flux()
    assert _relerr(c, d) < 1e-12


def test_graph_solve_matches_plain_launches(moc):
    """moc_solve on a non-default stream runs every iteration as one captured
    graph with an 8-byte residual read; on the default stream the same
    launches go one by one.  Both stop at the same iteration with the same
    flux (up to the order of FP64 atomic additions), and both match
    fixed-count iterations of moc_iterate."""
    import torch
    prob = P.small_lattice()
    plan = moc.Plan(prob)
    out = {}
    for mode in ("own", "current"):
        s = moc.Solver(plan, stream=mode)
        s.set_source(prob.q)
        phi, st = s.solve(tol=1e-9, max_iters=400, sweep_fp64=True)
        assert st["converged"]
        out[mode] = (phi, st)
        s.reset()
        s.iterate(st["iters"], sweep_fp64=True)
        np.testing.assert_allclose(s.flux(), phi, rtol=1e-12)
        s.close()
    torch.cuda.synchronize()
    assert out["own"][1]["iters"] == out["current"][1]["iters"]
    np.testing.assert_allclose(out["own"][0], out["current"][0], rtol=1e-12)
    assert out["own"][1]["sweep_ms_median"] > 0
