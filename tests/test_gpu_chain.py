"""GPU parity of the chain-line sweep (moc_solver_set_chain) against the
oracle's chain mode, and its invariants.

In chain mode every z-stack line is swept whole, from the z face it enters
through to the one it leaves through, the flux crossing the reflective side
faces within the sweep.  Tolerances as for the lagged sweep: the FP32 sweep
is held to 1e-5 max relative FSR error against the FP64 oracle.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_17743_amd import problems as P

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def moc():
    import torch
    assert torch.cuda.is_available()
    from paper_2503_17743_amd import moc as M
    M.lib()
    return M


def _chain_solver(moc, prob):
    plan = moc.Plan(prob)
    s = moc.Solver(plan)
    s.set_source(prob.q)
    s.set_chain(True)
    return plan, s


def _relerr(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def test_chain_fixed_iterations_match_oracle(moc, nthreads):
    """After 1, 2 and 5 source iterations the FSR fluxes and the leakage match
    the oracle's chain iterates, and every line piece is swept exactly once
    per sweep (the segment-group count of the lagged sweep)."""
    prob = P.small_lattice()
    plan, s = _chain_solver(moc, prob)
    om = O.Model(prob, n_threads=nthreads)
    for iters in (1, 2, 5):
        s.reset()
        print(f"chain small_lattice: {iters} iterations", flush=True)
        st = s.iterate(iters)
        ophi, ores = om.solve(tol=0.0, max_iters=iters, chain=True)
        assert _relerr(s.flux(), ophi) < TOL32, iters
        assert abs(st["leakage"] - ores["leakage"]) < TOL32 * ores["leakage"]
        assert st["link_errors"] == 0
        assert st["seg_group_updates"] == 2 * om.info["n_segments"] * prob.n_groups
        # per-sweep balance: sum W dpsi = sum W psi_in - sum W psi_out
        assert abs(st["balance_lhs"] - st["balance_rhs"]) < 1e-5 * abs(st["balance_rhs"])


def test_chain_iterates_differ_from_lagged(moc, nthreads):
    """The chain sweep is not the lagged one: after one iteration the lagged
    sweep's side-face fluxes are still zero and its flux is lower."""
    prob = P.small_lattice()
    plan, s = _chain_solver(moc, prob)
    s.iterate(1)
    chain = s.flux()
    s.set_chain(False)
    s.reset()
    s.iterate(1)
    lagged = s.flux()
    om = O.Model(prob, n_threads=nthreads)
    olag, _ = om.solve(tol=0.0, max_iters=1)
    assert _relerr(lagged, olag) < TOL32
    assert np.min(chain - lagged) >= 0.0 and _relerr(lagged, chain) > 1e-2


def test_chain_converged_matches_oracle(moc, nthreads):
    """Converged chain iteration: the oracle's fixed point to the FP32 bar,
    in fewer iterations than the lagged iteration needs, and the lagged
    iteration reaches the same flux."""
    prob = P.small_lattice()
    plan, s = _chain_solver(moc, prob)
    phi, st = s.solve(tol=1e-6, max_iters=500)
    om = O.Model(prob, n_threads=nthreads)
    ophi, ores = om.solve(tol=1e-11, max_iters=500, chain=True)
    assert st["converged"] and st["link_errors"] == 0, st
    assert _relerr(phi, ophi) < TOL32
    s.set_chain(False)
    phl, stl = s.solve(tol=1e-6, max_iters=500)
    assert stl["converged"] and _relerr(phl, ophi) < TOL32, stl
    assert st["iters"] < stl["iters"]
    assert abs(st["absorption"] + st["leakage"] - st["source"]) < 1e-5 * st["source"]


@pytest.mark.parametrize("tau,n_polar,n_layers", [(0.7, 6, 4), (3.0, 8, 5)])
def test_chain_slab_profile_closed_form(moc, tau, n_polar, n_layers):
    """Pure absorber in a slab (reflective sides, vacuum z): one chain sweep
    gives each layer the average of qhat (1 - e^{-Sigma_t z/|mu|}) over the
    discrete directions, z measured from each line's entry face."""
    H = 2.0
    sig = tau / H
    prob = P.pure_absorber(n_groups=1, sigma=(sig,), q=[1.0], bc=(1, 1, 1, 1, 0, 0), nx=1,
                           pitch=1.5, height=H, n_layers=n_layers, n_azim=8, n_polar=n_polar,
                           radial=0.05, axial=0.05, max_iters=1)
    plan, s = _chain_solver(moc, prob)
    s.iterate(1)
    phi = s.flux()[:, 0]
    q = O.Model(prob, trace=False).quadrature()
    c = np.abs(q["cot"])
    mu = c / np.sqrt(1 + c * c)
    w = q["dphi"][:, None] * q["wpol"][None, :]
    qhat = 1.0 / (4 * math.pi * sig)
    h = H / n_layers
    z = np.arange(n_layers + 1) * h

    def layer_mean(z0, z1):
        return 1 - mu / (sig * h) * (np.exp(-sig * z0 / mu) - np.exp(-sig * z1 / mu))

    exact = np.array([qhat * np.sum(w * (layer_mean(z[k], z[k + 1]) + layer_mean(H - z[k + 1], H - z[k])))
                      for k in range(n_layers)])
    np.testing.assert_allclose(phi, exact, rtol=TOL32)


def test_chain_lattice8_matches_oracle(moc, nthreads):
    """lattice8 (8x8 cells, 20 layers, 7 groups, 16 x 6 angles): three chain
    iterations against the oracle's."""
    prob = P.get("lattice8")
    plan, s = _chain_solver(moc, prob)
    print("chain lattice8: 3 iterations", flush=True)
    st = s.iterate(3)
    om = O.Model(prob, n_threads=nthreads)
    ophi, ores = om.solve(tol=0.0, max_iters=3, chain=True)
    assert _relerr(s.flux(), ophi) < TOL32
    assert st["link_errors"] == 0
    assert st["seg_group_updates"] == 2 * om.info["n_segments"] * prob.n_groups


def test_chain_window_sizes_agree(moc):
    """Every workgroup size of the per-lane sweep gives the same chain iterate
    (windows end at 2D segment boundaries; only the FP64 tally order moves)."""
    prob = P.small_lattice()
    plan, s = _chain_solver(moc, prob)
    ref = None
    for nt in (256, 512, 1024):
        try:
            s.set_window(nt)
        except moc.MocError:
            continue
        s.reset()
        s.iterate(2)
        phi = s.flux()
        if ref is None:
            ref = phi
        else:
            assert _relerr(phi, ref) < 1e-6, nt
    assert ref is not None


def test_chain_segments_cover_every_line(moc, nthreads):
    """A coarser problem whose cycles are cut into many segments (a line's
    reach is short against the cycle): still every line swept once, as the
    oracle's chain iterate."""
    prob = P.small_lattice(n=4, height=2.0, n_layers=2, n_azim=16, n_polar=6, radial=0.1, axial=0.25)
    plan = moc.Plan(prob)
    assert plan.info["n_chain_segments"] > 4 * 4
    s = moc.Solver(plan)
    s.set_source(prob.q)
    s.set_chain(True)
    st = s.iterate(3)
    om = O.Model(prob, n_threads=nthreads)
    ophi, ores = om.solve(tol=0.0, max_iters=3, chain=True)
    assert _relerr(s.flux(), ophi) < TOL32
    assert abs(st["leakage"] - ores["leakage"]) < TOL32 * ores["leakage"]
    assert st["seg_group_updates"] == 2 * om.info["n_segments"] * prob.n_groups
    assert st["link_errors"] == 0


def test_chain_only_solver(moc, nthreads):
    """A workspace without the boundary buffers gives a chain-only solver
    (split classes): the oracle's chain iterates, the full solver's results,
    and no way out of chain mode or into the hooks that need the buffers."""
    prob = P.small_lattice()
    plan = moc.Plan(prob)
    s = moc.Solver(plan, chain_only=True)
    assert s.workspace.numel() < plan.info["workspace_bytes"]
    s.set_source(prob.q)
    st = s.iterate(3)
    om = O.Model(prob, n_threads=nthreads)
    ophi, _ = om.solve(tol=0.0, max_iters=3, chain=True)
    assert _relerr(s.flux(), ophi) < TOL32
    assert st["seg_group_updates"] == 2 * om.info["n_segments"] * prob.n_groups
    full = moc.Solver(plan)
    full.set_source(prob.q)
    full.set_chain(2)
    full.iterate(3)
    assert _relerr(s.flux(), full.flux()) < 1e-6
    with pytest.raises(moc.MocError):
        s.set_chain(False)
    with pytest.raises(moc.MocError):
        s.boundary_flux(np.zeros(1, np.int64))
    # moc_solve (captured iterations) in the chain-only solver
    phi, stc = s.solve(tol=1e-6, max_iters=500)
    oconv, _ = om.solve(tol=1e-11, max_iters=500, chain=True)
    assert stc["converged"] and _relerr(phi, oconv) < TOL32


def test_chain_eigenvalue_matches_oracle(moc, nthreads):
    """Power iteration on k-eff with chain-line sweeps (chain-only solver) has
    the lagged iteration's fixed point: k and the flux shape within 1e-5 of
    the oracle's converged FP64 solution."""
    p = P.small_lattice()
    nsf, chi = P.fission_data(p)
    s = moc.Solver(moc.Plan(p), chain_only=True)
    s.set_source(p.q)
    _, _, st6 = s.solve_eigen(nsf, chi, tol=1e-6, max_iters=2000)
    assert st6["converged"]
    phi, k, st = s.solve_eigen(nsf, chi, tol=0.0, max_iters=600)
    om = O.Model(p, n_threads=nthreads)
    ophi, ok, ores = om.solve_eigen(nsf, chi, tol=1e-10, max_iters=5000)
    print(f"chain k {k:.8f} oracle {ok:.8f}, iterations to 1e-6 {st6['iters']}")
    assert abs(k - ok) < 1e-5 * ok
    a, b = phi / np.sum(phi), ophi / np.sum(ophi)
    m = b > 0
    assert np.max(np.abs(a[m] - b[m]) / b[m]) < 1e-5


@pytest.mark.parametrize("case", ["one_layer", "two_polar", "tall_narrow"])
def test_chain_degenerate_cases(moc, nthreads, case):
    """One axial layer; the minimal polar quadrature (one angle each way);
    a tall narrow box whose lines wrap round their short cycles many times
    before they reach the other z face (many passes past the cycle origin)."""
    if case == "one_layer":
        prob = P.small_lattice(seed=31, n_layers=1, height=1.0)
    elif case == "two_polar":
        prob = P.small_lattice(seed=32, n_polar=2)
    else:
        prob = P.small_lattice(seed=34, n=1, height=12.0, n_layers=6, n_azim=4, n_polar=4,
                               radial=0.1, axial=0.3)
    plan = moc.Plan(prob)
    s = moc.Solver(plan, chain_only=True)
    s.set_source(prob.q)
    st = s.iterate(2)
    om = O.Model(prob, n_threads=nthreads)
    ophi, ores = om.solve(tol=0.0, max_iters=2, chain=True)
    assert _relerr(s.flux(), ophi) < TOL32
    assert st["seg_group_updates"] == 2 * om.info["n_segments"] * prob.n_groups
    assert st["link_errors"] == 0


def test_solver_picks_chain_only_when_the_workspace_does_not_fit(moc):
    """lattice64 with half the axial spacing: the full workspace (about 428 GB)
    exceeds the GPU, so Solver(plan) makes a chain-only solver (about 7 GB)
    and sweeps it; chain_only=False refuses to allocate rather than fall back."""
    import torch
    prob = P.get("lattice64_fine")
    plan = moc.Plan(prob)
    free, _ = torch.cuda.mem_get_info()
    assert plan.info["workspace_bytes"] > free
    s = moc.Solver(plan)
    assert s.workspace.numel() < 16 * (1 << 30)
    with pytest.raises(moc.MocError):
        s.set_chain(False)
    s.close()
    del s
    torch.cuda.empty_cache()
    with pytest.raises(torch.OutOfMemoryError):
        moc.Solver(plan, chain_only=False)


def test_chain_rejections(moc):
    """Chain mode needs vacuum top and bottom faces, and in chain mode the
    FP64 sweep is refused rather than run lagged."""
    prob = P.config_plain()      # reflective on all faces
    plan = moc.Plan(prob)
    s = moc.Solver(plan)
    with pytest.raises(moc.MocError) as e:
        s.set_chain(True)
    assert e.value.code == moc.MOC_EINVAL
    prob = P.small_lattice()
    plan, s = _chain_solver(moc, prob)
    with pytest.raises(moc.MocError) as e:
        s.iterate(1, sweep_fp64=True)
    assert e.value.code == moc.MOC_EINVAL
    s.set_chain(False)
    s.iterate(1, sweep_fp64=True)
