"""Eigenvalue mode (power iteration on k-eff) on the GPU: the infinite-medium
multiplication factors, and the small heterogeneous lattice against the FP64
oracle iteration by iteration and converged."""
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


def _solver(moc, prob):
    s = moc.Solver(moc.Plan(prob))
    s.set_source(prob.q)
    return s


@pytest.mark.parametrize("fp64", [False, True])
def test_eigen_one_group_infinite_medium(moc, fp64):
    """k = nuSigma_f / (Sigma_t - Sigma_s) = 1.2, flat flux."""
    p = P.config_plain()
    s = _solver(moc, p)
    if fp64:
        phi, k, st = s.solve_eigen([[0.6]], [[1.0]], tol=1e-10, max_iters=3000, sweep_fp64=True)
        assert st["converged"]
    else:
        phi, k, st = s.solve_eigen([[0.6]], [[1.0]], tol=0.0, max_iters=3000)
    assert abs(k - 1.2) < (1e-8 if fp64 else 1e-5)
    np.testing.assert_allclose(phi / phi.mean(), 1.0, rtol=1e-8 if fp64 else 1e-5)


@pytest.mark.parametrize("fp64", [False, True])
def test_eigen_multigroup_infinite_medium(moc, fp64):
    """k = the eigenvalue of (diag Sigma_t - Sigma_s^T)^-1 chi nuSigma_f^T."""
    p = P.homogeneous(n_groups=4)
    nsf, chi = P.fission_data(p, k_target=1.05)
    s = _solver(moc, p)
    # the all-reflective medium converges slowly (lagged boundary flux): the
    # FP32 sweep, whose residual floor is near tol, runs a fixed 4000 iterations
    if fp64:
        phi, k, st = s.solve_eigen(nsf, chi, tol=1e-10, max_iters=5000, sweep_fp64=True)
        assert st["converged"]
    else:
        phi, k, st = s.solve_eigen(nsf, chi, tol=0.0, max_iters=4000)
    A = np.diag(p.sigma_t[0]) - p.sigma_s[0].T
    kref = max(np.linalg.eigvals(np.linalg.solve(A, np.outer(chi[0], nsf[0]))).real)
    assert abs(k - kref) < (1e-8 if fp64 else 1e-5) * kref
    spec = np.linalg.solve(A, chi[0])
    np.testing.assert_allclose(phi / phi[:, :1], np.tile(spec / spec[0], (p.n_fsr, 1)),
                               rtol=1e-7 if fp64 else 1e-5)


@pytest.mark.parametrize("fp64", [False, True])
def test_eigen_lattice_fixed_iterations_match_oracle(moc, nthreads, fp64):
    """The same 8 power iterations on the GPU and in the oracle: k and every
    FSR-group flux."""
    p = P.small_lattice()
    nsf, chi = P.fission_data(p)
    s = _solver(moc, p)
    om = O.Model(p, n_threads=nthreads)
    phi, k, st = s.solve_eigen(nsf, chi, tol=0.0, max_iters=8, sweep_fp64=fp64)
    assert st["iters"] == 8 and not st["converged"]
    ophi, ok, ores = om.solve_eigen(nsf, chi, tol=0.0, max_iters=8)
    print(f"fp64={fp64}: k {k:.10f} oracle {ok:.10f}")
    assert abs(k - ok) < (1e-11 if fp64 else 1e-6) * ok
    m = ophi > 0
    err = np.max(np.abs(phi[m] - ophi[m]) / ophi[m])
    assert err < (1e-10 if fp64 else 1e-5), err
    assert abs(st["residual"] - ores["residual"]) < (1e-6 if fp64 else 1e-3) * ores["residual"] + 1e-12


def test_eigen_lattice_converged_matches_oracle(moc, nthreads):
    """FP32 power iteration run to its floor (a fixed 600 iterations): k and
    the flux shape within 1e-5 of the oracle's converged FP64 solution; the
    FP32 run also stops by itself at tol 1e-6."""
    p = P.small_lattice()
    nsf, chi = P.fission_data(p)
    s = _solver(moc, p)
    _, _, st6 = s.solve_eigen(nsf, chi, tol=1e-6, max_iters=2000)
    assert st6["converged"]
    phi, k, st = s.solve_eigen(nsf, chi, tol=0.0, max_iters=600)
    om = O.Model(p, n_threads=nthreads)
    ophi, ok, ores = om.solve_eigen(nsf, chi, tol=1e-10, max_iters=5000)
    print(f"k {k:.8f} oracle {ok:.8f}, iterations {st['iters']} / {ores['iters']}")
    assert abs(k - ok) < 1e-5 * ok
    # the amplitude of an eigenvector is arbitrary: compare shapes
    a, b = phi / np.sum(phi), ophi / np.sum(ophi)
    m = b > 0
    assert np.max(np.abs(a[m] - b[m]) / b[m]) < 1e-5


def test_eigen_rejects_bad_input_and_fixed_source_still_works(moc):
    p = P.small_lattice()
    nsf, chi = P.fission_data(p)
    s = _solver(moc, p)
    with pytest.raises(moc.MocError):
        s.solve_eigen(np.zeros_like(nsf), chi)
    bad = chi.copy()
    bad[0, 0] = -1.0
    with pytest.raises(moc.MocError):
        s.solve_eigen(nsf, bad)
    s.solve_eigen(nsf, chi, tol=1e-4, max_iters=50)
    # the eigenvalue solve overwrote the source: set it again
    s.set_source(p.q)
    phi, st = s.solve(tol=1e-6, max_iters=500)
    ref = _solver(moc, p).solve(tol=1e-6, max_iters=500)[0]
    assert np.max(np.abs(phi - ref) / np.maximum(np.abs(ref), 1e-300)) < 1e-9
