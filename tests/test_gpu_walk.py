"""The two transport walks of the FP32 sweep (lockstep and per-lane) against
the FP64 oracle, and against each other.  Both give every line the same
pieces in the same order, so they differ only by the order of FP64 tally
additions (and, through it, rare FP32 roundings of the reduced source)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_17743_amd import problems as P

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
WALKS = ("lockstep", "lane")


@pytest.fixture(scope="module")
def moc():
    import torch
    assert torch.cuda.is_available()
    from paper_2503_17743_amd import moc as M
    M.lib()
    return M


def _relerr(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def _solver(moc, prob, walk):
    plan = moc.Plan(prob)
    s = moc.Solver(plan, fp64_boundary=False)
    s.set_source(prob.q)
    s.set_walk(walk)
    assert s.walk() == walk
    return plan, s


@pytest.mark.parametrize("walk", WALKS)
@pytest.mark.parametrize("case", ["small", "deep", "lattice8"])
def test_walk_fixed_iterations_match_oracle(moc, nthreads, walk, case):
    if case == "small":
        prob, iters = P.small_lattice(), (1, 5)
    elif case == "deep":
        # strided bundles (every 10th line) in several blocks
        prob, iters = P.small_lattice(seed=12, n=2, height=60.0, n_layers=60, n_groups=2, n_azim=4,
                                      n_polar=2, axial=0.1), (1, 4)
    else:
        prob, iters = P.config_lattice8(), (3,)
    plan, s = _solver(moc, prob, walk)
    om = O.Model(prob, n_threads=nthreads)
    for it in iters:
        s.reset()
        st = s.iterate(it)
        ophi, ores = om.solve(max_iters=it, tol=0.0)
        err = _relerr(s.flux(), ophi)
        print(f"{case} {walk} {it} iterations: max rel err {err:.3e}")
        assert err < TOL32, (case, walk, it, err)
        assert st["link_errors"] == 0
        assert st["seg_group_updates"] == 2 * om.info["n_segments"] * prob.n_groups
        assert abs(st["leakage"] - ores["leakage"]) <= 1e-5 * abs(ores["leakage"]) + 1e-30


@pytest.mark.parametrize("walk", WALKS)
def test_walk_sampled_sweep_matches_oracle(moc, walk):
    """One sweep of random bundles with random incoming flux and reduced
    source: outgoing flux and tallies of exactly those tracks."""
    prob = P.config_lattice8()
    plan, s = _solver(moc, prob, walk)
    om = O.Model(prob, trace=False)
    rng = np.random.default_rng(17)
    T, G = plan.info["tracks_per_wave"], prob.n_groups
    items = rng.choice(2 * plan.info["n_chunks"], size=300, replace=False)
    qhat = P.f32(rng.uniform(0.0, 0.2, size=(plan.info["n_fsr"], G)))
    psi_in = P.f32(rng.uniform(0.0, 0.5, size=(len(items), T, G)))
    acc, psi_out = s.sweep_items(items, qhat, psi_in)
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
    np.testing.assert_allclose(gpsi, opsi, rtol=2e-6, atol=2e-6 * np.abs(opsi).max())
    nz = np.abs(oacc) > 0
    assert (np.abs(acc[~nz]) == 0).all()
    np.testing.assert_allclose(acc, oacc, rtol=0, atol=1e-5 * np.abs(oacc).max())


def test_walks_agree(moc):
    """Same problem, same iterations: the walks' fluxes agree far inside the
    FP32 tolerance, and the same segment-group count is swept."""
    prob = P.config_lattice8()
    out = {}
    for walk in WALKS:
        plan, s = _solver(moc, prob, walk)
        st = s.iterate(6)
        out[walk] = (s.flux(), st["seg_group_updates"])
        s.close()
    assert out["lockstep"][1] == out["lane"][1]
    assert _relerr(out["lane"][0], out["lockstep"][0]) < 1e-6


def test_walk_selection(moc):
    """auto resolves to one of the two walks; explicit choices stick; bad
    values are rejected."""
    prob = P.small_lattice()
    plan = moc.Plan(prob)
    s = moc.Solver(plan, fp64_boundary=False)
    s.set_walk("auto")
    assert s.walk() in WALKS
    s.set_walk("lane")
    assert s.walk() == "lane"
    s.set_walk("lockstep")
    assert s.walk() == "lockstep"
    with pytest.raises(moc.MocError):
        moc._check(moc.lib().moc_solver_set_walk(s._h, 7))
