"""Seeded synthetic inputs for fixed-source 3D MOC problems.

This module only builds inputs: geometry records, tracking parameters,
multigroup cross sections and volumetric sources.  It performs none of the
transport method's arithmetic, so both the HIP library and the FP64 oracle can
be fed from it without sharing any part of the method.

Five named workloads stand in for the paper's C5G7-style pin-cell lattices
(whose evaluated nuclear data are not available): every value is synthetic and
drawn from ``numpy.random.default_rng(seed)``, then rounded to the nearest
float32 so that input rounding is never a source of disagreement between the
two implementations.

Material recipe (applies to every lattice workload): for each material and
group, Sigma_t ~ U[0.2, 2.0].  For each material and source group g_from the
total out-scatter is c * Sigma_t[g_from] with c ~ U[0.3, 0.9]; it is split over
destination groups g_to >= g_from (downscatter and self-scatter only) by
normalised U(0, 1] fractions.  Sources Q ~ U[0, 1] per (inclusion material,
group); the matrix material carries no source.

FSR numbering contract (used to lay the per-FSR source out):
  cell = cy * nx + cx
  local region = 2 * sector + (0 if inside the inclusion else 1) when the cell
                 has an inclusion (radius > 0), else local = sector
  radial region r = cell * regions_per_cell + local
  3D FSR j = r * n_layers + k   (k = axial layer, layer-fastest)
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

BC_VACUUM = 0
BC_REFLECTIVE = 1
# face order: x-, x+, y-, y+, z-, z+
ALL_REFLECTIVE = (1, 1, 1, 1, 1, 1)
REFLECTIVE_SIDES_VACUUM_Z = (1, 1, 1, 1, 0, 0)


def f32(a):
    """Round to the nearest float32 value and return float64 storage."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


@dataclasses.dataclass
class Problem:
    """One fixed-source problem: geometry + tracking + cross sections + source."""
    name: str
    # geometry
    nx: int
    ny: int
    pitch: float
    radius: float
    n_sectors: int
    height: float
    n_layers: int
    bc: tuple
    cell_material: np.ndarray          # int32 [ny*nx, 2] = {inside, outside}
    # tracking
    n_azim: int
    n_polar: int
    radial_spacing: float
    axial_spacing: float
    # cross sections
    n_groups: int
    sigma_t: np.ndarray                # float64 [M, G]
    sigma_s: np.ndarray                # float64 [M, G, G]  [m][g_from][g_to]
    # source per FSR
    q: np.ndarray                      # float64 [n_fsr, G]
    # solve controls
    tol: float = 1e-10
    max_iters: int = 2000
    seed: Optional[int] = None

    @property
    def n_materials(self) -> int:
        return int(self.sigma_t.shape[0])

    @property
    def regions_per_cell(self) -> int:
        return (2 if self.radius > 0 else 1) * self.n_sectors

    @property
    def n_regions(self) -> int:
        return self.nx * self.ny * self.regions_per_cell

    @property
    def n_fsr(self) -> int:
        return self.n_regions * self.n_layers

    def region_material(self) -> np.ndarray:
        """Material id of every radial region, following the numbering contract."""
        rc = self.regions_per_cell
        out = np.empty(self.n_regions, dtype=np.int32)
        for cell in range(self.nx * self.ny):
            for local in range(rc):
                if self.radius > 0:
                    inside = (local % 2) == 0
                else:
                    inside = False
                out[cell * rc + local] = self.cell_material[cell, 0 if inside else 1]
        return out

    def fsr_material(self) -> np.ndarray:
        return np.repeat(self.region_material(), self.n_layers)


def random_materials(rng: np.random.Generator, n_mat: int, n_groups: int):
    """Sigma_t and a downscatter-only Sigma_s with bounded out-scatter ratio."""
    sigma_t = f32(rng.uniform(0.2, 2.0, size=(n_mat, n_groups)))
    sigma_s = np.zeros((n_mat, n_groups, n_groups))
    for m in range(n_mat):
        for g in range(n_groups):
            c = rng.uniform(0.3, 0.9)
            frac = 1.0 - rng.uniform(0.0, 1.0, size=n_groups - g)   # in (0, 1]
            frac = frac / frac.sum()
            sigma_s[m, g, g:] = c * sigma_t[m, g] * frac
    sigma_s = f32(sigma_s)
    # float32 rounding may only move the ratio by ~1e-7; keep it strictly < 1
    assert (sigma_s.sum(axis=2) < sigma_t).all()
    return sigma_t, sigma_s


def _source_per_fsr(prob_geom: dict, region_mat: np.ndarray, q_mat: np.ndarray,
                    n_layers: int) -> np.ndarray:
    q_reg = q_mat[region_mat]                      # [n_regions, G]
    return np.repeat(q_reg, n_layers, axis=0)      # [n_fsr, G], layer fastest


def _lattice(name, seed, n, height, n_layers, n_mat, n_groups, n_azim, n_polar,
             radial, axial, tol=1e-10, max_iters=2000, bc=REFLECTIVE_SIDES_VACUUM_Z,
             pitch=1.0, radius=0.4, n_sectors=8) -> Problem:
    rng = np.random.default_rng(seed)
    sigma_t, sigma_s = random_materials(rng, n_mat, n_groups)
    cell_mat = np.zeros((n * n, 2), dtype=np.int32)
    if n_mat == 2:
        cell_mat[:, 0] = 1
    else:
        cell_mat[:, 0] = rng.integers(1, n_mat, size=n * n)
    q_mat = np.zeros((n_mat, n_groups))
    q_mat[1:] = f32(rng.uniform(0.0, 1.0, size=(n_mat - 1, n_groups)))
    p = Problem(name=name, nx=n, ny=n, pitch=pitch, radius=radius, n_sectors=n_sectors,
                height=float(height), n_layers=n_layers, bc=tuple(bc),
                cell_material=cell_mat, n_azim=n_azim, n_polar=n_polar,
                radial_spacing=radial, axial_spacing=axial, n_groups=n_groups,
                sigma_t=sigma_t, sigma_s=sigma_s, q=np.zeros(0), tol=tol,
                max_iters=max_iters, seed=seed)
    p.q = _source_per_fsr({}, p.region_material(), q_mat, n_layers)
    return p


def config_plain() -> Problem:
    """4x4x4 cm box, 2x2x2 cubic FSRs, one material, one group, reflective on
    all faces; 4 azimuthal x 2 polar angles, 0.5 cm radial and axial spacing.
    Closed form: phi = Q / (Sigma_t - Sigma_s) = 2.0 everywhere."""
    cell_mat = np.zeros((4, 2), dtype=np.int32)
    p = Problem(name="plain_box", nx=2, ny=2, pitch=2.0, radius=0.0, n_sectors=1,
                height=4.0, n_layers=2, bc=ALL_REFLECTIVE, cell_material=cell_mat,
                n_azim=4, n_polar=2, radial_spacing=0.5, axial_spacing=0.5,
                n_groups=1, sigma_t=np.array([[1.0]]), sigma_s=np.array([[[0.5]]]),
                q=np.ones((8, 1)), tol=1e-10, max_iters=2000, seed=None)
    return p


def config_lattice8() -> Problem:
    """8x8 pin cells (pitch 1 cm, inclusion r = 0.4 cm, 8 sectors x 2 rings),
    20 cm tall in 20 layers, 2 materials, 7 groups; reflective sides, vacuum
    top/bottom; 16 azimuthal x 6 polar, 0.05 cm radial, 0.2 cm axial."""
    return _lattice("lattice8", 2, 8, 20.0, 20, 2, 7, 16, 6, 0.05, 0.2)


def config_lattice32() -> Problem:
    """32x32 lattice of the same cell, 100 cm / 100 layers, 4 materials, 7
    groups, 32 azimuthal x 6 polar, 0.05 / 0.25 cm."""
    return _lattice("lattice32", 3, 32, 100.0, 100, 4, 7, 32, 6, 0.05, 0.25)


def config_lattice64() -> Problem:
    """Largest single-GPU case: 64x64 lattice, 200 cm / 200 layers, 4 materials,
    7 groups, 64 azimuthal x 8 polar, 0.03 / 0.1 cm; 50 source iterations."""
    return _lattice("lattice64", 5, 64, 200.0, 200, 4, 7, 64, 8, 0.03, 0.1,
                    max_iters=50)


def config_lattice64_fine() -> Problem:
    """lattice64 with half the axial ray spacing (0.05 cm): twice the 3D
    tracks, whose two boundary angular-flux buffers (about 420 GB) exceed one
    GPU's memory; a chain-line sweep needs none of them."""
    return _lattice("lattice64_fine", 5, 64, 200.0, 200, 4, 7, 64, 8, 0.03, 0.05,
                    max_iters=50)


def small_lattice(seed=11, n=3, height=3.0, n_layers=3, n_groups=3, n_mat=3,
                  n_azim=8, n_polar=4, radial=0.2, axial=0.3,
                  bc=REFLECTIVE_SIDES_VACUUM_Z, n_sectors=4, radius=0.35,
                  tol=1e-10, max_iters=2000) -> Problem:
    """A reduced lattice of the same construction, sized for seconds of oracle
    time while still spanning many waves and ragged stacks."""
    return _lattice(f"small_n{n}_s{seed}", seed, n, height, n_layers, n_mat, n_groups,
                    n_azim, n_polar, radial, axial, tol=tol, max_iters=max_iters,
                    bc=bc, n_sectors=n_sectors, radius=radius)


def homogeneous(material_seed=2, n_groups=7, nx=2, pitch=1.0, height=2.0, n_layers=2,
                n_azim=8, n_polar=4, radial=0.1, axial=0.2, radius=0.4, n_sectors=8,
                q_value=None) -> Problem:
    """One material everywhere (the lattice recipe's matrix/inclusion split is
    kept as region structure, but both regions carry material 0), reflective on
    all faces, uniform source: an infinite homogeneous medium."""
    rng = np.random.default_rng(material_seed)
    sigma_t, sigma_s = random_materials(rng, 1, n_groups)
    q_g = f32(rng.uniform(0.2, 1.0, size=n_groups)) if q_value is None else \
        np.full(n_groups, float(q_value))
    cell_mat = np.zeros((nx * nx, 2), dtype=np.int32)
    p = Problem(name="homogeneous", nx=nx, ny=nx, pitch=pitch, radius=radius,
                n_sectors=n_sectors, height=height, n_layers=n_layers, bc=ALL_REFLECTIVE,
                cell_material=cell_mat, n_azim=n_azim, n_polar=n_polar,
                radial_spacing=radial, axial_spacing=axial, n_groups=n_groups,
                sigma_t=sigma_t, sigma_s=sigma_s, q=np.zeros(0), tol=1e-11, max_iters=5000)
    p.q = np.tile(q_g, (p.n_fsr, 1))
    return p


def fission_data(prob: Problem, fissile=(0,), seed=7, k_target=1.1):
    """Synthetic fission data for eigenvalue mode (no evaluated nuclear data):
    nu_sigma_f [M, G] and chi [M, G].  Fissile materials produce neutrons in
    proportion to a random profile rising towards the slow groups; chi is a
    fast spectrum (weight 2^-g, normalised).  The profile is scaled so that
    the material's own infinite-medium multiplication factor is k_target,
    which keeps lattice eigenvalues near one."""
    rng = np.random.default_rng(seed)
    M, G = prob.n_materials, prob.n_groups
    chi = np.tile(2.0 ** -np.arange(G), (M, 1))
    chi /= chi.sum(axis=1, keepdims=True)
    nsf = np.zeros((M, G))
    for m in fissile:
        shape = rng.uniform(0.2, 1.0, size=G) * np.linspace(0.5, 1.5, G)
        A = np.diag(prob.sigma_t[m]) - prob.sigma_s[m].T
        kinf = float(shape @ np.linalg.solve(A, chi[m]))
        nsf[m] = shape * (k_target / kinf)
    return nsf, chi


def pure_absorber(n_groups=2, sigma=(0.7, 1.3), q=None, bc=(0, 0, 0, 0, 0, 0), **kw) -> Problem:
    """Homogeneous box with no scattering (a pure absorber), vacuum by default."""
    nx = kw.pop("nx", 2)
    p = Problem(name="absorber", nx=nx, ny=nx, pitch=kw.pop("pitch", 1.0),
                radius=kw.pop("radius", 0.0), n_sectors=kw.pop("n_sectors", 1),
                height=kw.pop("height", 2.0), n_layers=kw.pop("n_layers", 2), bc=tuple(bc),
                cell_material=np.zeros((nx * nx, 2), dtype=np.int32),
                n_azim=kw.pop("n_azim", 4), n_polar=kw.pop("n_polar", 2),
                radial_spacing=kw.pop("radial", 0.25), axial_spacing=kw.pop("axial", 0.25),
                n_groups=n_groups, sigma_t=np.array([list(sigma)]),
                sigma_s=np.zeros((1, n_groups, n_groups)), q=np.zeros(0), tol=1e-12,
                max_iters=kw.pop("max_iters", 200))
    assert not kw, kw
    p.q = np.zeros((p.n_fsr, n_groups)) if q is None else np.tile(np.asarray(q, float), (p.n_fsr, 1))
    return p


# --------------------------------------------------------------------------
# serving stream
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    problem: Problem
    arrival_s: float


def serving_stream(n_requests=512, seed=4, rate_per_s=None, sizes=(4, 8, 16),
                   layers=(10, 50), groups=(1, 7), azim=(8, 32), polar=(2, 4, 6),
                   radial=0.05, axial=0.2, tol=1e-6) -> List[Request]:
    """Independent fixed-source lattice problems of random size (the problems
    depend only on seed) with Poisson arrival times (exponential gaps of mean
    1/rate from a generator of their own; rate None = all at t=0)."""
    rng = np.random.default_rng(seed)
    probs = []
    for i in range(n_requests):
        n = int(rng.choice(sizes))
        k = int(rng.integers(layers[0], layers[1] + 1))
        g = int(rng.integers(groups[0], groups[1] + 1))
        a = int(rng.choice(np.arange(azim[0], azim[1] + 1, 4)))
        pp = int(rng.choice(polar))
        sub_seed = int(rng.integers(0, 2**31 - 1))
        probs.append(_lattice(f"req{i}", sub_seed, n, float(k), k, 2, g, a, pp, radial, axial,
                              tol=tol, max_iters=1000))
    return with_arrivals(probs, rate_per_s, seed)


def with_arrivals(problems, rate_per_s, seed=4) -> List[Request]:
    """Poisson arrivals for a list of problems (rate None: all at t=0)."""
    if not rate_per_s:
        return [Request(p, 0.0) for p in problems]
    gaps = np.random.default_rng([seed, 1]).exponential(1.0 / rate_per_s, len(problems))
    return [Request(p, float(t)) for p, t in zip(problems, np.cumsum(gaps))]


CONFIGS = {
    "plain_box": config_plain,
    "lattice8": config_lattice8,
    "lattice32": config_lattice32,
    "lattice64": config_lattice64,
    "lattice64_fine": config_lattice64_fine,
}


def get(name: str) -> Problem:
    return CONFIGS[name]()
