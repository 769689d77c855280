"""Thin ctypes binding of libmoc.so (the C ABI in include/moc.h).

Argument marshalling only: every step of the transport path runs in the HIP
library.  PyTorch provides device memory (the solver workspace is a torch
uint8 tensor) and the stream (torch's current stream).  There is no fallback:
if the library is missing or cannot be loaded, the import of the library
raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmoc.so")

MOC_OK, MOC_EINVAL, MOC_ENOMEM, MOC_EDEVICE, MOC_ENOTCONV, MOC_EBUSY = 0, -1, -2, -3, -4, -5


class MocError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"moc error {code}: {msg}")
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("pitch", C.c_double),
                ("inclusion_radius", C.c_double), ("n_sectors", C.c_int),
                ("height", C.c_double), ("n_layers", C.c_int), ("bc", C.c_int * 6),
                ("cell_material", C.POINTER(C.c_int))]


class Tracking(C.Structure):
    _fields_ = [("n_azim", C.c_int), ("n_polar", C.c_int), ("radial_spacing", C.c_double),
                ("axial_spacing", C.c_double)]


class XS(C.Structure):
    _fields_ = [("n_groups", C.c_int), ("n_materials", C.c_int),
                ("sigma_t", C.POINTER(C.c_double)), ("sigma_s", C.POINTER(C.c_double))]


class PlanInfo(C.Structure):
    _fields_ = [("n_fsr", C.c_longlong), ("n_regions", C.c_longlong),
                ("n_2d_tracks", C.c_longlong), ("n_2d_segments", C.c_longlong),
                ("n_stacks", C.c_longlong), ("n_3d_tracks", C.c_longlong),
                ("n_chunks", C.c_longlong), ("n_groups", C.c_int), ("tracks_per_wave", C.c_int),
                ("dz", C.c_double), ("workspace_bytes", C.c_size_t), ("psi_bytes", C.c_size_t),
                ("workspace_bytes_fp64", C.c_size_t), ("line_stride", C.c_int),
                ("workspace_bytes_chain", C.c_size_t), ("n_chain_segments", C.c_longlong),
                ("n_chain_items", C.c_longlong)]


class StoreInfo(C.Structure):
    _fields_ = [("units_stored", C.c_longlong), ("units_total", C.c_longlong),
                ("wave_steps_stored", C.c_ulonglong), ("wave_steps_total", C.c_ulonglong),
                ("bytes_used", C.c_size_t), ("bytes_all", C.c_size_t)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iters", C.c_int), ("sweep_fp64", C.c_int),
                ("exp_mode", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("residual", C.c_double), ("balance_lhs", C.c_double),
                ("balance_rhs", C.c_double), ("absorption", C.c_double), ("leakage", C.c_double),
                ("source", C.c_double), ("seg_group_updates", C.c_ulonglong),
                ("link_errors", C.c_ulonglong), ("sweep_ms_median", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
VP = C.c_void_p


def lib():
    """Load libmoc.so; raises if it is not built (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # torch carries its own HIP runtime under the same soname as the one the
    # library links against.  Loading torch first makes the dynamic loader bind
    # the library to that copy, so the process holds one HIP runtime and the
    # workspace pointers and streams torch hands over are valid in the library.
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    sig = {
        "moc_last_error": ([], C.c_char_p),
        "moc_plan_create": ([C.POINTER(Geometry), C.POINTER(Tracking), C.POINTER(XS), C.POINTER(VP)], C.c_int),
        "moc_plan_query": ([VP, C.POINTER(PlanInfo)], C.c_int),
        "moc_plan_destroy": ([VP], None),
        "moc_plan_quadrature": ([VP] + [VP] * 5, C.c_int),
        "moc_plan_tracks2d": ([VP] + [VP] * 6, C.c_int),
        "moc_plan_stacks": ([VP] + [VP] * 3, C.c_int),
        "moc_plan_segments2d": ([VP] + [VP] * 3, C.c_int),
        "moc_plan_chain": ([VP] + [VP] * 6, C.c_int),
        "moc_plan_chunk": ([VP, C.c_longlong, C.POINTER(C.c_longlong), C.POINTER(C.c_int)], C.c_int),
        "moc_solver_create": ([VP, VP, C.c_size_t, VP, C.POINTER(VP)], C.c_int),
        "moc_solver_destroy": ([VP], None),
        "moc_set_source": ([VP, VP, C.c_size_t], C.c_int),
        "moc_solve": ([VP, C.POINTER(SolveOpts), C.POINTER(Stats)], C.c_int),
        "moc_reset": ([VP], C.c_int),
        "moc_solve_eigen": ([VP, VP, VP, C.POINTER(SolveOpts), C.POINTER(C.c_double), C.POINTER(Stats)], C.c_int),
        "moc_solver_set_walk": ([VP, C.c_int], C.c_int),
        "moc_solver_walk": ([VP, C.POINTER(C.c_int)], C.c_int),
        "moc_solver_store_segments": ([VP, VP, C.c_size_t, C.POINTER(StoreInfo)], C.c_int),
        "moc_solver_set_schedule": ([VP, C.c_int, C.c_int], C.c_int),
        "moc_solver_set_window": ([VP, C.c_int], C.c_int),
        "moc_solver_set_bundles": ([VP, C.c_int], C.c_int),
        "moc_solver_set_chain": ([VP, C.c_int], C.c_int),
        "moc_solver_window": ([VP, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "moc_iterate": ([VP, C.c_int, C.POINTER(SolveOpts), C.POINTER(Stats)], C.c_int),
        "moc_get_flux": ([VP, VP, C.c_size_t], C.c_int),
        "moc_get_volumes": ([VP, VP, C.c_size_t], C.c_int),
        "moc_flux_device_ptr": ([VP, C.POINTER(VP)], C.c_int),
        "moc_sweep_items": ([VP, C.c_longlong, VP, VP, VP, C.c_int, VP, VP], C.c_int),
        "moc_trace_tracks": ([VP, C.c_longlong, VP, C.c_int, VP, VP, VP], C.c_int),
        "moc_get_reduced_source": ([VP, C.c_int, VP, C.c_size_t], C.c_int),
        "moc_get_boundary_flux": ([VP, C.c_longlong, VP, VP], C.c_int),
        "moc_server_create": ([VP, C.c_size_t, C.c_int, VP, C.POINTER(VP)], C.c_int),
        "moc_server_destroy": ([VP], None),
        "moc_server_arena_overhead": ([C.c_int, C.POINTER(C.c_size_t)], C.c_int),
        "moc_eval_attenuation": ([VP, C.c_longlong, C.c_int, VP], C.c_int),
        "moc_eval_attenuation_noalloc": ([VP, C.c_longlong, C.c_int, VP], C.c_int),
        "moc_server_query": ([VP, C.c_ulonglong, C.POINTER(C.c_int)], C.c_int),
        "moc_server_set_fill": ([VP, C.c_longlong], C.c_int),
        "moc_server_submit": ([VP, VP, VP, C.POINTER(SolveOpts), C.POINTER(C.c_ulonglong)], C.c_int),
        "moc_server_step": ([VP, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
        "moc_server_poll": ([VP, C.c_ulonglong, C.POINTER(Stats), VP, C.c_size_t], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return _lib


def _check(rc, allow=()):
    if rc != MOC_OK and rc not in allow:
        raise MocError(rc, lib().moc_last_error().decode())
    return rc


def _p(a: np.ndarray):
    return a.ctypes.data_as(VP)


class Plan:
    """Host plan of one problem (problems.Problem-like object)."""

    def __init__(self, prob):
        self.prob = prob
        self._cm = np.ascontiguousarray(prob.cell_material, dtype=np.int32)
        self._st = np.ascontiguousarray(prob.sigma_t, dtype=np.float64)
        self._ss = np.ascontiguousarray(prob.sigma_s, dtype=np.float64)
        g = Geometry(prob.nx, prob.ny, prob.pitch, prob.radius, prob.n_sectors, prob.height,
                     prob.n_layers)
        for i in range(6):
            g.bc[i] = int(prob.bc[i])
        g.cell_material = self._cm.ctypes.data_as(C.POINTER(C.c_int))
        t = Tracking(prob.n_azim, prob.n_polar, prob.radial_spacing, prob.axial_spacing)
        x = XS(prob.n_groups, self._st.shape[0], self._st.ctypes.data_as(C.POINTER(C.c_double)),
               self._ss.ctypes.data_as(C.POINTER(C.c_double)))
        h = VP()
        _check(lib().moc_plan_create(C.byref(g), C.byref(t), C.byref(x), C.byref(h)))
        self._h = h
        inf = PlanInfo()
        _check(lib().moc_plan_query(h, C.byref(inf)))
        self.info = {f: getattr(inf, f) for f, _ in PlanInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().moc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def quadrature(self):
        A2, P = self.prob.n_azim // 2, self.prob.n_polar
        out = dict(phi=np.zeros(A2), dphi=np.zeros(A2), spacing=np.zeros(A2),
                   cot=np.zeros((A2, P)), weight=np.zeros((A2, P)))
        _check(lib().moc_plan_quadrature(self._h, *[_p(out[k]) for k in
                                                     ("phi", "dphi", "spacing", "cot", "weight")]))
        return out

    def tracks2d(self):
        n = self.info["n_2d_tracks"]
        out = dict(xy=np.zeros((n, 4)), length=np.zeros(n), azim=np.zeros(n, np.int32),
                   link=np.zeros((n, 2), np.int64), chain=np.zeros(n), sigma=np.zeros(n, np.int32))
        _check(lib().moc_plan_tracks2d(self._h, *[_p(out[k]) for k in
                                                   ("xy", "length", "azim", "link", "chain", "sigma")]))
        return out

    def stacks(self):
        ns = self.info["n_stacks"]
        z, lo, cnt = np.zeros(ns), np.zeros(ns, np.int64), np.zeros(ns, np.int64)
        _check(lib().moc_plan_stacks(self._h, _p(z), _p(lo), _p(cnt)))
        return z, lo, cnt

    def segments2d(self):
        n = self.info["n_2d_segments"]
        pos, reg = np.zeros(n), np.zeros(n, np.int32)
        first = np.zeros(self.info["n_2d_tracks"] + 1, np.int64)
        _check(lib().moc_plan_segments2d(self._h, _p(pos), _p(reg), _p(first)))
        return pos, reg, first

    def chain(self):
        """Segments of the chain-line sweep (moc_plan_chain)."""
        ns, ni = self.info["n_chain_segments"], self.info["n_chain_items"]
        out = dict(first=np.zeros(ns + 1, np.int64), k=np.zeros(ns, np.int32), nk=np.zeros(ns, np.int32),
                   lc=np.zeros(ns), code=np.zeros(ni, np.int32), u=np.zeros(ni))
        _check(lib().moc_plan_chain(self._h, *[_p(out[x]) for x in ("first", "k", "nk", "lc", "code", "u")]))
        return out

    def chunk(self, c: int):
        ft, nt = C.c_longlong(), C.c_int()
        _check(lib().moc_plan_chunk(self._h, int(c), C.byref(ft), C.byref(nt)))
        return ft.value, nt.value


class Solver:
    """A plan bound to a device workspace (torch uint8 tensor) and a stream.

    stream="own" (default) gives the solver a non-default torch stream of its
    own, on which moc_solve runs each iteration as one captured HIP graph;
    stream="current" uses torch's current stream (plain launches when that is
    the default stream)."""

    def __init__(self, plan: Plan, device="cuda", workspace=None, fp64_boundary=None, walk="auto",
                 stream="own", chain_only="auto"):
        """chain_only: True gives a solver without boundary buffers (chain-line
        sweeps only); "auto" does so when the full workspace would not fit in
        the device's free memory and the plan allows chain sweeps; False never."""
        import torch
        self.plan = plan
        self.info = plan.info
        if chain_only == "auto":
            chain_only = False
            if workspace is None and plan.info["workspace_bytes_chain"]:
                free, _ = torch.cuda.mem_get_info(torch.device(device))
                chain_only = plan.info["workspace_bytes"] + (1 << 30) > free
        if chain_only:
            # no boundary buffers: the solver sweeps chain lines only
            if not plan.info["workspace_bytes_chain"]:
                raise MocError(MOC_EINVAL, "the plan has no chain-line sweep (vacuum top and bottom)")
            nbytes = int(plan.info["workspace_bytes_chain"])
        else:
            if fp64_boundary is None:   # FP64 boundary flux when it costs < 1 GiB
                fp64_boundary = plan.info["workspace_bytes_fp64"] < (1 << 30)
            nbytes = int(plan.info["workspace_bytes_fp64" if fp64_boundary else "workspace_bytes"])
        if workspace is None:
            workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self.workspace = workspace
        base = workspace.data_ptr()
        aligned = (base + 255) & ~255
        avail = workspace.numel() - (aligned - base)
        if stream == "own":
            # the workspace was allocated on the current stream: order the
            # solver's stream after it
            self.stream = torch.cuda.Stream(workspace.device)
            self.stream.wait_stream(torch.cuda.current_stream(workspace.device))
        else:
            self.stream = torch.cuda.current_stream(workspace.device)
        h = VP()
        _check(lib().moc_solver_create(plan._h, VP(aligned), avail, VP(self.stream.cuda_stream),
                                       C.byref(h)))
        self._h = h
        self.n_fsr = plan.info["n_fsr"]
        self.G = plan.info["n_groups"]
        self._store = None
        if walk != "auto":
            self.set_walk(walk)

    def close(self):
        if getattr(self, "_h", None):
            # the workspace returns to torch's allocator with the tensor: let
            # the solver's stream finish with it first
            self.stream.synchronize()
            lib().moc_solver_destroy(self._h)
            self._h = None
            self._store = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_source(self, q):
        q = np.ascontiguousarray(q, dtype=np.float64)
        _check(lib().moc_set_source(self._h, _p(q), q.size))

    def solve(self, tol=1e-10, max_iters=1000, sweep_fp64=False, exp_mode=0):
        o = SolveOpts(float(tol), int(max_iters), int(sweep_fp64), int(exp_mode))
        st = Stats()
        rc = _check(lib().moc_solve(self._h, C.byref(o), C.byref(st)), allow=(MOC_ENOTCONV,))
        d = st.as_dict()
        d["converged"] = rc == MOC_OK
        return self.flux(), d

    def solve_eigen(self, nu_sigma_f, chi, tol=1e-6, max_iters=1000, sweep_fp64=False):
        """Power iteration on k-eff (moc_solve_eigen): (phi [n_fsr][G], not
        normalised; k; stats).  Overwrites the fixed source."""
        nsf = np.ascontiguousarray(nu_sigma_f, dtype=np.float64)
        ch = np.ascontiguousarray(chi, dtype=np.float64)
        if nsf.shape != ch.shape or nsf.ndim != 2 or nsf.shape[1] != self.G:
            raise ValueError("nu_sigma_f and chi must both be [M][G]")
        o = SolveOpts(float(tol), int(max_iters), int(sweep_fp64), 0)
        k = C.c_double()
        st = Stats()
        rc = _check(lib().moc_solve_eigen(self._h, _p(nsf), _p(ch), C.byref(o), C.byref(k), C.byref(st)),
                    allow=(MOC_ENOTCONV,))
        d = st.as_dict()
        d["converged"] = rc == MOC_OK
        return self.flux(), k.value, d

    def reset(self):
        _check(lib().moc_reset(self._h))

    WALKS = {"auto": 0, "lockstep": 1, "lane": 2}

    def set_walk(self, walk="auto"):
        """Transport walk of the FP32 one-chunk sweep: auto, lockstep or lane (per-lane)."""
        _check(lib().moc_solver_set_walk(self._h, self.WALKS[walk]))

    ORDERS = {"longest_first": 0, "natural": 1, "alternating": 2}

    def set_schedule(self, order="longest_first", persistent=False):
        """Work-unit schedule (section 4.3): longest_first, natural or
        alternating (decreasing work in groups of the resident workgroup
        count, every other group reversed); persistent: a grid of resident
        workgroups sweeping units b, b + grid, ...  Drops any store."""
        _check(lib().moc_solver_set_schedule(self._h, self.ORDERS[order], int(bool(persistent))))
        self._store = None

    def store_segments(self, fraction=0.8, max_bytes=None):
        """Stored-segment sweep (section 4.2): keep the pieces of the units
        with the largest footprint in a device buffer of at most `fraction`
        of the free device memory (or max_bytes), replayed by later sweeps.
        fraction=0 drops the store.  Returns the store info as a dict."""
        import torch
        inf = StoreInfo()
        if fraction <= 0 and not max_bytes:
            _check(lib().moc_solver_store_segments(self._h, None, 0, C.byref(inf)))
            self._store = None
            return {f: getattr(inf, f) for f, _ in StoreInfo._fields_}
        dev = self.workspace.device
        # count first with a small buffer, then size the store
        n_units = 2 * self.info["n_2d_tracks"]
        small = torch.empty(n_units * 24 + 4096, dtype=torch.uint8, device=dev)
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        _check(lib().moc_solver_store_segments(self._h, VP((small.data_ptr() + 255) & ~255),
                                                small.numel() - 256, C.byref(inf)))
        self.stream.synchronize()
        del small
        torch.cuda.empty_cache()
        free, _ = torch.cuda.mem_get_info(dev)
        cap = int(fraction * free) if fraction > 0 else 0
        if max_bytes:
            cap = min(cap, int(max_bytes)) if cap else int(max_bytes)
        nbytes = min(int(inf.bytes_all), cap)
        self._store = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        self.stream.wait_stream(torch.cuda.current_stream(dev))
        base = (self._store.data_ptr() + 255) & ~255
        _check(lib().moc_solver_store_segments(self._h, VP(base), nbytes, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in StoreInfo._fields_}

    BUNDLES = {"auto": -1, "static": 0, "dynamic": 1}

    def set_bundles(self, mode="auto"):
        """How a workgroup's waves share a window's bundles: static (wave w
        takes w, w + waves, ...), dynamic (the next untaken one), or auto."""
        _check(lib().moc_solver_set_bundles(self._h, self.BUNDLES[mode]))

    def set_chain(self, on=True):
        """Chain-line sweeping (moc_solver_set_chain): every line swept whole
        from the z face it enters through to the one it leaves through, the
        flux crossing reflective side faces within the sweep."""
        _check(lib().moc_solver_set_chain(self._h, 1 if on else 0))

    def set_window(self, threads=0):
        """Workgroup size of the per-lane sweep: 0 (automatic), 256, 512, 1024."""
        _check(lib().moc_solver_set_window(self._h, int(threads)))
        self._store = None

    def window(self):
        """(workgroup threads, 2D segments per window) of the per-lane sweep."""
        t, w = C.c_int(), C.c_int()
        _check(lib().moc_solver_window(self._h, C.byref(t), C.byref(w)))
        return t.value, w.value

    def walk(self):
        w = C.c_int()
        _check(lib().moc_solver_walk(self._h, C.byref(w)))
        return "lockstep" if w.value == 1 else "lane"

    def iterate(self, n, sweep_fp64=False, exp_mode=0, stats=True):
        o = SolveOpts(0.0, 1, int(sweep_fp64), int(exp_mode))
        st = Stats()
        _check(lib().moc_iterate(self._h, int(n), C.byref(o), C.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def flux(self):
        out = np.zeros((self.n_fsr, self.G))
        _check(lib().moc_get_flux(self._h, _p(out), out.size))
        return out

    def volumes(self):
        out = np.zeros(self.n_fsr)
        _check(lib().moc_get_volumes(self._h, _p(out), out.size))
        return out

    def flux_device_ptr(self) -> int:
        p = VP()
        _check(lib().moc_flux_device_ptr(self._h, C.byref(p)))
        return p.value

    def sweep_items(self, items, qhat, psi_in, sweep_fp64=False):
        items = np.ascontiguousarray(items, dtype=np.int64)
        qhat = np.ascontiguousarray(qhat, dtype=np.float64)
        T = self.info["tracks_per_wave"]
        psi_in = np.ascontiguousarray(psi_in, dtype=np.float64).reshape(len(items), T, self.G)
        acc = np.zeros((self.n_fsr, self.G))
        psi_out = np.zeros((len(items), T, self.G))
        _check(lib().moc_sweep_items(self._h, len(items), _p(items), _p(qhat), _p(psi_in),
                                     int(sweep_fp64), _p(acc), _p(psi_out)))
        return acc, psi_out

    def reduced_source(self, fp64=False):
        """qhat [n_fsr][G] of the last source update, as the sweep read it."""
        out = np.zeros((self.n_fsr, self.G))
        _check(lib().moc_get_reduced_source(self._h, int(bool(fp64)), _p(out), out.size))
        return out

    def boundary_flux(self, slots):
        """Incoming flux [n][G] the next sweep reads for directed slots 2*track+dir."""
        slots = np.ascontiguousarray(slots, dtype=np.int64)
        out = np.zeros((len(slots), self.G))
        _check(lib().moc_get_boundary_flux(self._h, len(slots), _p(slots), _p(out)))
        return out

    def trace_tracks(self, track_ids, cap=4096):
        ids = np.ascontiguousarray(track_ids, dtype=np.int64)
        fsr = np.zeros((len(ids), cap), np.int32)
        ln = np.zeros((len(ids), cap))
        cnt = np.zeros(len(ids), np.int32)
        _check(lib().moc_trace_tracks(self._h, len(ids), _p(ids), int(cap), _p(fsr), _p(ln), _p(cnt)))
        return [(fsr[i, :min(cnt[i], cap)].copy(), ln[i, :min(cnt[i], cap)].copy(), int(cnt[i]))
                for i in range(len(ids))]


class Server:
    """Continuous-batching server on a device arena (torch uint8 tensor) and
    its own non-default stream (so the batched step can be graph-captured)."""

    def __init__(self, arena_bytes, max_slots=64, device="cuda", fill_units=None):
        import torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device=self.device)
        torch.cuda.synchronize(self.device)
        base = self.arena.data_ptr()
        aligned = (base + 255) & ~255
        h = VP()
        _check(lib().moc_server_create(VP(aligned), self.arena.numel() - (aligned - base),
                                       int(max_slots), VP(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self._shape = {}
        if fill_units is not None:      # None: the library's default fill target
            _check(lib().moc_server_set_fill(self._h, int(fill_units)))

    @staticmethod
    def overhead_bytes(max_slots=64) -> int:
        b = C.c_size_t()
        _check(lib().moc_server_arena_overhead(int(max_slots), C.byref(b)))
        return b.value

    def close(self):
        if getattr(self, "_h", None):
            lib().moc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, plan: Plan, q, tol=1e-6, max_iters=1000) -> int:
        q = np.ascontiguousarray(q, dtype=np.float64)
        o = SolveOpts(float(tol), int(max_iters), 0, 0)
        t = C.c_ulonglong()
        _check(lib().moc_server_submit(self._h, plan._h, _p(q), C.byref(o), C.byref(t)))
        self._shape[t.value] = (plan.info["n_fsr"], plan.info["n_groups"])
        return t.value

    def step(self):
        na, nq = C.c_int(), C.c_int()
        _check(lib().moc_server_step(self._h, C.byref(na), C.byref(nq)))
        return na.value, nq.value

    def done(self, ticket) -> bool:
        d = C.c_int()
        _check(lib().moc_server_query(self._h, C.c_ulonglong(ticket), C.byref(d)))
        return bool(d.value)

    def poll(self, ticket):
        """None while queued or running; else (flux, stats) and the request is released."""
        if not self.done(ticket):
            return None
        shape = self._shape[ticket]
        flux = np.empty(shape)
        st = Stats()
        rc = lib().moc_server_poll(self._h, C.c_ulonglong(ticket), C.byref(st), _p(flux), flux.size)
        if rc == MOC_EBUSY:
            return None
        _check(rc, allow=(MOC_ENOTCONV,))
        del self._shape[ticket]
        d = st.as_dict()
        d["converged"] = rc == MOC_OK
        return flux, d


def solve(prob, tol=None, max_iters=None, sweep_fp64=False, exp_mode=0):
    """Plan, bind and solve one problem; returns (phi [n_fsr, G], stats)."""
    plan = Plan(prob)
    s = Solver(plan)
    s.set_source(prob.q)
    return s.solve(tol=prob.tol if tol is None else tol,
                   max_iters=prob.max_iters if max_iters is None else max_iters,
                   sweep_fp64=sweep_fp64, exp_mode=exp_mode)


def eval_attenuation(tau, exp_mode=0):
    """The sweep's FP32 F(tau) = 1 - exp(-tau), evaluated on the device."""
    t = np.ascontiguousarray(tau, dtype=np.float32)
    out = np.empty_like(t)
    _check(lib().moc_eval_attenuation(_p(t), t.size, int(exp_mode), _p(out)))
    return out
