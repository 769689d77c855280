"""CPU checks of the chain-line sweep's plan: the segments of the directed 2D
cycles, with each item's per-stack line range (the entry-distance window the
sweep clips every stack to), sweep every directed 3D line exactly once, and
each segment's items are consecutive units of one directed cycle."""
import numpy as np
import pytest

from paper_2503_17743_amd import moc
from paper_2503_17743_amd import problems as P


CASES = {
    "small_lattice": lambda: P.small_lattice(),
    "many_segments": lambda: P.small_lattice(n=4, height=2.0, n_layers=2, n_azim=16, n_polar=6,
                                             radial=0.1, axial=0.25),
    "lines_lap_cycles": lambda: P.small_lattice(seed=34, n=1, height=12.0, n_layers=6, n_azim=4,
                                                n_polar=4, radial=0.1, axial=0.3),
    "lattice8": lambda: P.get("lattice8"),
}


def _line_ranges(u, k, nk, lc, c, d, lt, z0, cnt, dz, H):
    """Lines [lo, hi] of a stack (cot c, unit direction d, lowest line at z0
    on the 2D track's start) that entered the box within segment k of nk of a
    cycle of length lc, at an entry distance from the unit's unrolled start u
    in (u - B, u - A]."""
    ce = -c if d else c
    zs = z0 + c * (lt if d else 0.0)            # z of line 0 where the unit starts
    kk = np.rint(lc * abs(c) / dz)
    sp = lc / kk
    a, b = np.floor(k * kk / nk) * sp, np.floor((k + 1) * kk / nk) * sp
    x0, x1 = u - b, u - a
    if ce > 0:      # rising: entered through the bottom, z / ce before
        lo, hi = np.floor((ce * x0 - zs) / dz) + 1, np.floor((ce * x1 - zs) / dz)
    else:           # falling: through the top, (H - z) / |ce| before
        lo, hi = np.ceil((H + ce * x1 - zs) / dz), np.ceil((H + ce * x0 - zs) / dz) - 1
    return int(max(lo, 0)), int(min(hi, cnt - 1))


@pytest.mark.parametrize("case", sorted(CASES))
def test_chain_segments_sweep_every_line_once(case):
    prob = CASES[case]()
    plan = moc.Plan(prob)
    info = plan.info
    assert info["n_chain_segments"] > 0
    ch = plan.chain()
    q = plan.quadrature()
    tr = plan.tracks2d()
    zeta, ilo, cnt = plan.stacks()
    Pn, dz, H = prob.n_polar, info["dz"], prob.height
    trk_off = np.concatenate([[0], np.cumsum(cnt)])
    n3d = int(trk_off[-1])
    assert n3d == info["n_3d_tracks"]
    # difference array over directed slots 2 * (trk_off[s] + i) + dir, per direction
    diff = np.zeros((2, n3d + 1), np.int32)
    link = tr["link"].reshape(-1)
    for sg in range(info["n_chain_segments"]):
        i0, i1 = int(ch["first"][sg]), int(ch["first"][sg + 1])
        assert i1 > i0
        k, nk, lc = int(ch["k"][sg]), int(ch["nk"][sg]), float(ch["lc"][sg])
        for i in range(i0, i1):
            code, u = int(ch["code"][i]), float(ch["u"][i])
            if i > i0:
                # consecutive units of one directed cycle, positions in step
                prev = int(ch["code"][i - 1])
                assert link[prev] == code
                step = tr["length"][prev >> 1]
                assert abs(u - (float(ch["u"][i - 1]) + step)) < 1e-6 * max(1.0, lc)
            t, d = code >> 1, code & 1
            for n in range(Pn):
                s = t * Pn + n
                if cnt[s] == 0:
                    continue
                c = q["cot"][tr["azim"][t], n]
                z0 = zeta[s] + ilo[s] * dz
                lo, hi = _line_ranges(u, k, nk, lc, c, d, tr["length"][t], z0, int(cnt[s]), dz, H)
                if hi >= lo:
                    diff[d, trk_off[s] + lo] += 1
                    diff[d, trk_off[s] + hi + 1] -= 1
    cover = np.cumsum(diff[:, :n3d], axis=1)
    assert cover.min() == 1 and cover.max() == 1, (int(cover.min()), int(cover.max()))
