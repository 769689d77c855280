"""CPU checks of the C ABI: the library loads and exports every declared
symbol, argument validation, and the host planner's laydown (quadrature,
2D links, chain phases, z-stack table) equals the oracle's exactly."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_17743_amd import moc
from paper_2503_17743_amd import problems as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"MOC_API\s+[\w\s\*]+?\b(moc_\w+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 20
    L = C.CDLL(moc.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_library_shares_torchs_hip_runtime():
    """Loading the library before anything imported torch must still leave one
    HIP runtime in the process, torch's (two copies cannot share device
    pointers or streams)."""
    import subprocess
    import sys
    code = ("from paper_2503_17743_amd import moc\n"
            "moc.lib()\n"
            "import torch, os\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "libs = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l})\n"
            "tdir = os.path.realpath(os.path.dirname(torch.__file__))\n"
            "assert len(libs) == 1, libs\n"
            "assert os.path.realpath(libs[0]).startswith(tdir), libs\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]


def test_chain_only_workspace_size():
    """A chain-only solver's workspace is the full one without the two
    boundary buffers (which the layout puts last); plans without vacuum top
    and bottom faces have none."""
    for prob in (P.small_lattice(), P.get("lattice8")):
        info = moc.Plan(prob).info
        assert info["workspace_bytes_chain"] == info["workspace_bytes"] - info["psi_bytes"]
        assert info["psi_bytes"] >= 2 * 2 * info["n_3d_tracks"] * prob.n_groups * 4
    assert moc.Plan(P.config_plain()).info["workspace_bytes_chain"] == 0


def _plan_err(prob):
    with pytest.raises(moc.MocError) as e:
        moc.Plan(prob)
    return e.value.code


@pytest.mark.parametrize("field,value", [
    ("n_azim", 6), ("n_azim", 0), ("n_polar", 3), ("radial_spacing", 0.0),
    ("axial_spacing", -1.0), ("radius", 0.5), ("radius", -0.1), ("n_sectors", 3),
])
def test_plan_rejects_invalid_geometry_and_tracking(field, value):
    p = P.small_lattice()
    setattr(p, field, value)
    assert _plan_err(p) == moc.MOC_EINVAL


def test_plan_rejects_invalid_xs_and_bc():
    p = P.small_lattice()
    p.sigma_t = p.sigma_t.copy()
    p.sigma_t[0, 0] = 0.0
    assert _plan_err(p) == moc.MOC_EINVAL
    p = P.small_lattice()
    p.sigma_s = p.sigma_s.copy()
    p.sigma_s[1, 0, 1] = -1e-3
    assert _plan_err(p) == moc.MOC_EINVAL
    p = P.small_lattice()
    p.sigma_s = p.sigma_s.copy()
    p.sigma_s[0, 0, 0] = p.sigma_t[0, 0]          # ratio >= 1
    assert _plan_err(p) == moc.MOC_EINVAL
    p = P.small_lattice()
    p.cell_material = p.cell_material.copy()
    p.cell_material[0, 0] = 7
    assert _plan_err(p) == moc.MOC_EINVAL
    p = P.small_lattice()
    p.bc = (1, 1, 2, 1, 0, 0)
    assert _plan_err(p) == moc.MOC_EINVAL
    p = P.small_lattice(n_groups=3)
    p.n_groups = 65
    assert _plan_err(p) == moc.MOC_EINVAL


def test_plan_error_text_is_reported():
    p = P.small_lattice()
    p.n_polar = 5
    with pytest.raises(moc.MocError) as e:
        moc.Plan(p)
    assert "n_polar" in str(e.value)


LAYDOWN_CASES = [P.config_plain, P.small_lattice, P.config_lattice8,
                 lambda: P.small_lattice(seed=3, n=4, n_azim=12, n_polar=6, radial=0.13,
                                         axial=0.17, height=2.3, n_layers=5, n_sectors=16),
                 lambda: P.homogeneous()]


@pytest.mark.parametrize("maker", LAYDOWN_CASES)
def test_planner_laydown_equals_oracle(maker):
    prob = maker()
    pl = moc.Plan(prob)
    om = O.Model(prob, trace=False)
    assert pl.info["n_fsr"] == om.info["n_fsr"]
    assert pl.info["n_2d_tracks"] == om.info["n_2d_tracks"]
    assert pl.info["n_3d_tracks"] == om.info["n_3d_tracks"]
    qp, qo = pl.quadrature(), om.quadrature()
    for k in ("phi", "dphi", "spacing", "cot", "weight"):
        np.testing.assert_allclose(qp[k], qo[k], rtol=1e-14, atol=1e-15)
    tp, to = pl.tracks2d(), om.tracks2d()
    np.testing.assert_allclose(tp["xy"], to["xy"], atol=1e-12)
    np.testing.assert_array_equal(tp["link"], to["link"])
    np.testing.assert_array_equal(tp["sigma"], to["sigma"])
    np.testing.assert_allclose(tp["chain"], to["chain"], atol=1e-9)
    zp, lp, cp = pl.stacks()
    zo, lo, co = om.stacks()
    np.testing.assert_array_equal(cp, co)
    np.testing.assert_array_equal(lp, lo)
    np.testing.assert_allclose(zp, zo, atol=1e-9)


def test_planner_2d_segments_tile_each_track():
    prob = P.config_lattice8()
    pl = moc.Plan(prob)
    pos, reg, first = pl.segments2d()
    t2 = pl.tracks2d()
    assert first[-1] == len(pos)
    assert (np.diff(first) >= 1).all()
    # positions start at 0 and increase strictly inside each track
    for t in range(0, len(first) - 1, 37):
        p = pos[first[t]:first[t + 1]]
        assert p[0] == 0.0 and (np.diff(p) > 0).all() and p[-1] < t2["length"][t]
        r = reg[first[t]:first[t + 1]]
        assert (r[1:] != r[:-1]).all()


def test_chunks_cover_stacks_exactly():
    prob = P.small_lattice()
    pl = moc.Plan(prob)
    T = pl.info["tracks_per_wave"]
    # lanes = (line, group chunk), chunks of at most 8 groups
    assert T == 64 // -(-prob.n_groups // 8)
    covered = 0
    prev_end = 0
    for c in range(pl.info["n_chunks"]):
        ft, nt = pl.chunk(c)
        assert 1 <= nt <= T
        assert ft == prev_end
        prev_end = ft + nt
        covered += nt
    assert covered == pl.info["n_3d_tracks"]


def test_workspace_footprint_grows_with_problem():
    a = moc.Plan(P.small_lattice()).info
    b = moc.Plan(P.config_lattice8()).info
    assert 0 < a["workspace_bytes"] < b["workspace_bytes"]
    assert b["psi_bytes"] == pytest.approx(2 * 2 * b["n_3d_tracks"] * b["n_groups"] * 4, rel=1e-3)


def test_null_and_invalid_arguments_are_rejected_without_a_device():
    """Entry points check their arguments before any device work: NULL
    handles and out-of-range values give MOC_EINVAL (no GPU is needed)."""
    L = moc.lib()
    opts = moc.SolveOpts(1e-6, 10, 0, 0)
    k = C.c_double()
    nsf = np.ones(4)
    assert L.moc_solve_eigen(None, moc._p(nsf), moc._p(nsf), C.byref(opts), C.byref(k), None) == moc.MOC_EINVAL
    assert L.moc_solver_set_walk(None, 0) == moc.MOC_EINVAL
    w = C.c_int()
    assert L.moc_solver_walk(None, C.byref(w)) == moc.MOC_EINVAL
    assert L.moc_server_set_fill(None, 1) == moc.MOC_EINVAL
    done = C.c_int()
    assert L.moc_server_query(None, C.c_ulonglong(1), C.byref(done)) == moc.MOC_EINVAL
    assert L.moc_server_step(None, None, None) == moc.MOC_EINVAL
    b = C.c_size_t()
    assert L.moc_server_arena_overhead(0, C.byref(b)) == moc.MOC_EINVAL
    assert L.moc_server_arena_overhead(64, C.byref(b)) == moc.MOC_OK and b.value > 0
    bad_tau = np.array([-1.0], np.float32)
    out = np.zeros(1, np.float32)
    assert L.moc_eval_attenuation(moc._p(bad_tau), 1, 0, moc._p(out)) == moc.MOC_EINVAL
    assert L.moc_eval_attenuation(moc._p(np.array([0.5], np.float32)), 1, 2, moc._p(out)) == moc.MOC_EINVAL
    assert len(L.moc_last_error().decode()) > 0
