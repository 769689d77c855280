"""ctypes binding of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The product path (the HIP library and its
Python binding) never imports, links or runs anything in this directory.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
# the mutation tests point this at an oracle built with a planted mistake
_LIB_OVERRIDE = os.environ.get("MOC_ORACLE_LIB")


def build(verbose=False, path=LIB_PATH, mutation=0) -> str:
    """Compile the oracle with gcc (plain C11 + OpenMP); mutation > 0 plants
    one of the mistakes listed in oracle.c (mutation tests only)."""
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           f"-DORC_MUTATION={int(mutation)}", "-o", path + ".tmp", os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(path + ".tmp", path)
    return path


class _Problem(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("pitch", C.c_double), ("radius", C.c_double),
                ("n_sectors", C.c_int), ("height", C.c_double), ("n_layers", C.c_int),
                ("bc", C.c_int * 6), ("cell_material", C.POINTER(C.c_int)),
                ("n_azim", C.c_int), ("n_polar", C.c_int), ("radial_spacing", C.c_double),
                ("axial_spacing", C.c_double), ("n_groups", C.c_int), ("n_materials", C.c_int),
                ("sigma_t", C.POINTER(C.c_double)), ("sigma_s", C.POINTER(C.c_double))]


class _Info(C.Structure):
    _fields_ = [("n_fsr", C.c_longlong), ("n_regions", C.c_longlong),
                ("n_2d_tracks", C.c_longlong), ("n_3d_tracks", C.c_longlong),
                ("n_segments", C.c_longlong), ("n_cycles", C.c_longlong),
                ("dz", C.c_double), ("traced", C.c_int)]


class _Result(C.Structure):
    _fields_ = [("iters", C.c_int), ("residual", C.c_double), ("leakage", C.c_double),
                ("balance_lhs", C.c_double), ("balance_rhs", C.c_double),
                ("absorption", C.c_double), ("source", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        src = os.path.join(HERE, "oracle.c")
        if _LIB_OVERRIDE:
            L = C.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
                build()
            L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.orc_gauss_legendre.argtypes = [C.c_int, P(C.c_double), P(C.c_double)]
        L.orc_build.argtypes = [P(_Problem), C.c_int, C.c_int, P(C.c_void_p)]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_get_info.argtypes = [C.c_void_p, P(_Info)]
        L.orc_get_quadrature.argtypes = [C.c_void_p] + [C.c_void_p] * 9
        L.orc_get_tracks2d.argtypes = [C.c_void_p] + [C.c_void_p] * 7
        L.orc_get_stacks.argtypes = [C.c_void_p] + [C.c_void_p] * 3
        L.orc_trace_track.argtypes = [C.c_void_p, C.c_longlong, C.c_void_p, C.c_void_p, C.c_longlong]
        L.orc_trace_track.restype = C.c_longlong
        L.orc_track_info.argtypes = [C.c_void_p, C.c_longlong, C.c_void_p, C.c_void_p]
        L.orc_volumes.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_segment_counts.argtypes = [C.c_void_p, C.c_void_p]
        L.orc_solve.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_void_p,
                                C.c_void_p, P(_Result)]
        L.orc_solve_ex.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_int, C.c_int, C.c_int,
                                   C.c_void_p, C.c_void_p, P(_Result)]
        L.orc_chain_info.argtypes = [C.c_void_p, P(C.c_longlong), P(C.c_longlong)]
        L.orc_solve_eigen.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int,
                                      C.c_void_p, P(C.c_double), C.c_void_p, P(_Result)]
        L.orc_sweep_sample.argtypes = [C.c_void_p, C.c_longlong, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_entry_vacuum.argtypes = [C.c_void_p, C.c_longlong, C.c_int]
        L.orc_sample_path_length.argtypes = [C.c_void_p, C.c_longlong, C.c_void_p, C.c_void_p,
                                             C.c_void_p]
        L.orc_track_weight.argtypes = [C.c_void_p, C.c_longlong]
        L.orc_track_weight.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def gauss_legendre(n: int):
    mu = np.zeros(n)
    w = np.zeros(n)
    rc = lib().orc_gauss_legendre(n, mu.ctypes.data_as(C.POINTER(C.c_double)),
                                  w.ctypes.data_as(C.POINTER(C.c_double)))
    assert rc == 0
    return mu, w


class Model:
    """Oracle model of one problem (laydown, stacks and optionally traced segments)."""

    def __init__(self, prob, trace=True, n_threads=0, overrides=None):
        self.prob = prob
        kw = dict(nx=prob.nx, ny=prob.ny, pitch=prob.pitch, radius=prob.radius,
                  n_sectors=prob.n_sectors, height=prob.height, n_layers=prob.n_layers,
                  n_azim=prob.n_azim, n_polar=prob.n_polar,
                  radial_spacing=prob.radial_spacing, axial_spacing=prob.axial_spacing,
                  n_groups=prob.n_groups, n_materials=prob.n_materials)
        if overrides:
            kw.update(overrides)
        self._cm = np.ascontiguousarray(prob.cell_material, dtype=np.int32)
        self._st = np.ascontiguousarray(prob.sigma_t, dtype=np.float64)
        self._ss = np.ascontiguousarray(prob.sigma_s, dtype=np.float64)
        p = _Problem()
        for k, v in kw.items():
            setattr(p, k, v)
        for i in range(6):
            p.bc[i] = int(prob.bc[i])
        p.cell_material = self._cm.ctypes.data_as(C.POINTER(C.c_int))
        p.sigma_t = self._st.ctypes.data_as(C.POINTER(C.c_double))
        p.sigma_s = self._ss.ctypes.data_as(C.POINTER(C.c_double))
        self._p = p
        h = C.c_void_p()
        rc = lib().orc_build(C.byref(p), 1 if trace else 0, int(n_threads), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle build failed: {rc}")
        self._h = h
        info = _Info()
        lib().orc_get_info(h, C.byref(info))
        self.info = {f: getattr(info, f) for f, _ in _Info._fields_}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    # ---- introspection ---------------------------------------------------
    def quadrature(self):
        A2, P = self.prob.n_azim // 2, self.prob.n_polar
        out = dict(phi=np.zeros(A2), dphi=np.zeros(A2), spacing=np.zeros(A2),
                   nx=np.zeros(A2, np.int32), ny=np.zeros(A2, np.int32), mu=np.zeros(P),
                   wpol=np.zeros(P), cot=np.zeros((A2, P)), weight=np.zeros((A2, P)))
        lib().orc_get_quadrature(self._h, *[_ptr(out[k]) for k in
                                            ("phi", "dphi", "spacing", "nx", "ny", "mu", "wpol",
                                             "cot", "weight")])
        return out

    def tracks2d(self):
        n = self.info["n_2d_tracks"]
        out = dict(xy=np.zeros((n, 4)), length=np.zeros(n), azim=np.zeros(n, np.int32),
                   faces=np.zeros((n, 2), np.int32), link=np.zeros((n, 2), np.int64),
                   chain=np.zeros(n), sigma=np.zeros(n, np.int32))
        lib().orc_get_tracks2d(self._h, *[_ptr(out[k]) for k in
                                          ("xy", "length", "azim", "faces", "link", "chain",
                                           "sigma")])
        return out

    def stacks(self):
        ns = self.info["n_2d_tracks"] * self.prob.n_polar
        z = np.zeros(ns)
        lo = np.zeros(ns, np.int64)
        cnt = np.zeros(ns, np.int64)
        lib().orc_get_stacks(self._h, _ptr(z), _ptr(lo), _ptr(cnt))
        return z, lo, cnt

    def trace(self, track: int):
        cap = 1 << 16
        f = np.zeros(cap, np.int32)
        l = np.zeros(cap)
        n = lib().orc_trace_track(self._h, int(track), _ptr(f), _ptr(l), cap)
        if n < 0 or n > cap:
            raise ValueError("trace failed")
        return f[:n].copy(), l[:n].copy()

    def track_info(self, track: int):
        p = np.zeros(6)
        s = np.zeros(2, np.int64)
        rc = lib().orc_track_info(self._h, int(track), _ptr(p), _ptr(s))
        if rc != 0:
            raise ValueError("track_info failed")
        return p[:3], p[3:], s

    def sample_path_length(self, tracks, wl=None):
        """sum of W l per FSR over the listed tracks (one direction each);
        accumulates into wl when given."""
        tracks = np.ascontiguousarray(tracks, dtype=np.int64)
        if wl is None:
            wl = np.zeros(self.info["n_fsr"])
        nseg = C.c_longlong(0)
        rc = lib().orc_sample_path_length(self._h, len(tracks), _ptr(tracks), _ptr(wl),
                                          C.byref(nseg))
        if rc != 0:
            raise ValueError("sample_path_length failed")
        return wl

    def entry_vacuum(self, tracks, dirs):
        """Boolean per directed track: it enters through a vacuum face."""
        out = np.zeros(len(tracks), bool)
        for i, (t, d) in enumerate(zip(tracks, dirs)):
            r = lib().orc_entry_vacuum(self._h, int(t), int(d))
            if r < 0:
                raise ValueError(f"entry_vacuum failed for track {t} dir {d}")
            out[i] = r == 1
        return out

    def weight(self, track: int) -> float:
        return lib().orc_track_weight(self._h, int(track))

    def segment_counts(self):
        c = np.zeros(self.info["n_3d_tracks"], np.int64)
        assert lib().orc_segment_counts(self._h, _ptr(c)) == 0
        return c

    def volumes(self):
        v = np.zeros(self.info["n_fsr"])
        assert lib().orc_volumes(self._h, _ptr(v)) == 0
        return v

    # ---- solves -----------------------------------------------------------
    def solve(self, q=None, tol=None, max_iters=None, chain=False, inner=1):
        """Source iteration (see orc_solve_ex): chain=False lags the boundary
        flux one sweep (inner sweeps per source iteration), chain=True sweeps
        whole chains of reflected tracks."""
        prob = self.prob
        q = np.ascontiguousarray(prob.q if q is None else q, dtype=np.float64)
        tol = prob.tol if tol is None else tol
        max_iters = prob.max_iters if max_iters is None else max_iters
        phi = np.zeros((self.info["n_fsr"], prob.n_groups))
        hist = np.zeros(max_iters)
        r = _Result()
        rc = lib().orc_solve_ex(self._h, _ptr(q), float(tol), int(max_iters), int(bool(chain)),
                                int(inner), _ptr(phi), _ptr(hist), C.byref(r))
        if rc != 0:
            raise ValueError(f"oracle solve failed: {rc}")
        res = {f: getattr(r, f) for f, _ in _Result._fields_}
        res["residual_history"] = hist[:r.iters].copy()
        return phi, res

    def chain_info(self):
        """(number of chains of directed tracks, longest chain in tracks)."""
        nh, ml = C.c_longlong(), C.c_longlong()
        rc = lib().orc_chain_info(self._h, C.byref(nh), C.byref(ml))
        if rc != 0:
            raise ValueError(f"oracle chain_info failed: {rc}")
        return nh.value, ml.value

    def solve_eigen(self, nu_sigma_f, chi, tol=1e-8, max_iters=1000):
        """Power iteration on k-eff (see orc_solve_eigen); returns
        (phi [n_fsr][G] unnormalised, k, result dict with residual_history)."""
        G = self.prob.n_groups
        nsf = np.ascontiguousarray(nu_sigma_f, dtype=np.float64).reshape(-1, G)
        ch = np.ascontiguousarray(chi, dtype=np.float64).reshape(-1, G)
        phi = np.zeros((self.info["n_fsr"], G))
        hist = np.zeros(max_iters)
        k = C.c_double()
        r = _Result()
        rc = lib().orc_solve_eigen(self._h, _ptr(nsf), _ptr(ch), float(tol), int(max_iters), _ptr(phi),
                                   C.byref(k), _ptr(hist), C.byref(r))
        if rc != 0:
            raise ValueError(f"oracle eigenvalue solve failed: {rc}")
        res = {f: getattr(r, f) for f, _ in _Result._fields_}
        res["residual_history"] = hist[:r.iters].copy()
        return phi, k.value, res

    def sweep_sample(self, tracks, dirs, qhat, psi_in):
        tracks = np.ascontiguousarray(tracks, dtype=np.int64)
        dirs = np.ascontiguousarray(dirs, dtype=np.int32)
        qhat = np.ascontiguousarray(qhat, dtype=np.float64)
        psi_in = np.ascontiguousarray(psi_in, dtype=np.float64)
        G = self.prob.n_groups
        acc = np.zeros((self.info["n_fsr"], G))
        psi_out = np.zeros((len(tracks), G))
        nseg = C.c_longlong(0)
        rc = lib().orc_sweep_sample(self._h, len(tracks), _ptr(tracks), _ptr(dirs), _ptr(qhat),
                                    _ptr(psi_in), _ptr(acc), _ptr(psi_out), C.byref(nseg))
        if rc != 0:
            raise ValueError("sweep_sample failed")
        return acc, psi_out, nseg.value
