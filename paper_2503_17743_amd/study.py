"""Precision and scale studies on the large lattices; one JSON line each.

  python -m paper_2503_17743_amd.study precision [--workload lattice32] [--iters 20]
      The same iterate of the FP32 sweep (stable and naive 1 - exp) and of the
      FP64 sweep from phi = 0; per-FSR-group relative error of each FP32 variant
      against the FP64 sweep.
  python -m paper_2503_17743_amd.study scale [--workload lattice64] [--iters 50]
      FP32 source iterations of the whole problem: time per sweep, residual
      history and the neutron balance of the last iteration.
  python -m paper_2503_17743_amd.study eigen [--workload lattice8] [--iters 2000] [--chain]
      Power iteration on k-eff (synthetic fission data, fissile inclusions)
      to 1e-6: k, iterations and time per iteration (--chain: chain-line sweeps).
  python -m paper_2503_17743_amd.study exp [--workload lattice8] [--iters 10]
      Stored-segment sweep and work-unit schedules: median sweep time of the
      on-the-fly sweep under each schedule and of the stored-segment sweep.
  python -m paper_2503_17743_amd.study window [--workload lattice32] [--iters 5]
      Median sweep time of the per-lane sweep for each workgroup size
      (256, 512, 1024 threads) with the largest window its LDS holds.
  python -m paper_2503_17743_amd.study bundles [--workload lattice32] [--iters 5]
      Median sweep time with static and with dynamic assignment of a window's
      bundles to the waves, for each workgroup size, in interleaved rounds.
  python -m paper_2503_17743_amd.study chain [--workload lattice8] [--iters 5] [--tol 1e-6]
      Lagged against chain-line sweeping: median sweep time of each, and (with
      --tol > 0) the iterations and time each takes to converge.
  python -m paper_2503_17743_amd.study chain_only [--workload lattice64] [--iters 10]
      A chain-only solver (no boundary buffers): workspace size, sweep time
      and residual history.

Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import moc, problems as P


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _rel_stats(phi, ref):
    m = np.abs(ref) > 0
    r = np.abs(phi[m] - ref[m]) / np.abs(ref[m])
    return {"max": float(r.max()), "p999": float(np.percentile(r, 99.9)),
            "p50": float(np.percentile(r, 50)), "n": int(m.sum())}


def precision(name, iters, fp64_boundary=None):
    import torch
    prob = P.get(name)
    plan = moc.Plan(prob)
    if fp64_boundary is None:
        free, _ = torch.cuda.mem_get_info()
        fp64_boundary = plan.info["workspace_bytes_fp64"] < 0.8 * free
    s = moc.Solver(plan, fp64_boundary=fp64_boundary)
    s.set_source(prob.q)
    runs = {}
    for label, kw in (("fp64_sweep", dict(sweep_fp64=True)), ("fp32_stable", dict()),
                      ("fp32_naive_exp", dict(exp_mode=1))):
        _log(f"precision {name}: {label}, {iters} iterations ...")
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.iterate(iters, **kw)
        torch.cuda.synchronize()
        runs[label] = (s.flux(), st, time.perf_counter() - t0)
    if fp64_boundary:
        # the production configuration: FP32 sweep with FP32 boundary storage
        s.close()
        del s
        torch.cuda.empty_cache()
        s = moc.Solver(plan, fp64_boundary=False)
        s.set_source(prob.q)
        _log(f"precision {name}: fp32_stable with FP32 boundary storage ...")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.iterate(iters)
        torch.cuda.synchronize()
        runs["fp32_stable_fp32_boundary"] = (s.flux(), st, time.perf_counter() - t0)
    ref = runs["fp64_sweep"][0]
    out = {"study": "precision", "workload": name, "iterations": iters,
           "fp64_boundary_storage": bool(fp64_boundary),
           "seg_group_updates_per_sweep": runs["fp32_stable"][1]["seg_group_updates"]}
    for label, (phi, st, t) in runs.items():
        d = {"sweep_ms_median": st["sweep_ms_median"], "wall_s": t, "residual": st["residual"],
             "balance_rel": abs(st["balance_lhs"] - st["balance_rhs"]) / max(abs(st["balance_rhs"]), 1e-300)}
        if label != "fp64_sweep":
            d["rel_err_vs_fp64_sweep"] = _rel_stats(phi, ref)
        out[label] = d
    s.close()
    return out


def scale(name, iters, walk="auto"):
    import torch
    prob = P.get(name)
    t0 = time.perf_counter()
    plan = moc.Plan(prob)
    t_plan = time.perf_counter() - t0
    _log(f"scale {name}: planned in {t_plan:.1f} s, workspace {plan.info['workspace_bytes'] / 1e9:.1f} GB")
    s = moc.Solver(plan, fp64_boundary=False, walk=walk)
    s.set_source(prob.q)
    torch.cuda.synchronize()
    hist, sweep_ms = [], []
    t0 = time.perf_counter()
    st = None
    for k in range(iters):
        st = s.iterate(1)
        hist.append(st["residual"])
        sweep_ms.append(st["sweep_ms_median"])
        _log(f"scale {name}: iteration {k + 1}/{iters} residual {st['residual']:.3e} "
             f"sweep {st['sweep_ms_median']:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    segg = st["seg_group_updates"]
    med = float(np.median(sweep_ms))
    out = {"study": "scale", "workload": name, "iterations": iters, "plan_s": t_plan,
           "n_fsr": plan.info["n_fsr"], "n_3d_tracks": plan.info["n_3d_tracks"],
           "workspace_bytes": plan.info["workspace_bytes"],
           "seg_group_updates_per_sweep": segg, "sweep_ms_median": med, "walk": s.walk(),
           "seg_group_per_s_sweep": segg / (med * 1e-3),
           "seg_group_per_s_wall": segg * iters / wall, "wall_s": wall,
           "residual_history": hist, "link_errors": st["link_errors"],
           "balance_rel": abs(st["balance_lhs"] - st["balance_rhs"]) / max(abs(st["balance_rhs"]), 1e-300)}
    s.close()
    return out


def eigen(name, tol=1e-6, max_iters=2000, walk="auto", chain=False):
    """Power iteration on k-eff of a lattice with synthetic fission data
    (fissile inclusion material): k, iterations, time per iteration; with
    chain=True in a chain-only solver (chain-line sweeps)."""
    import torch
    prob = P.get(name)
    nsf, chi = P.fission_data(prob)
    plan = moc.Plan(prob)
    s = moc.Solver(plan, fp64_boundary=False, walk=walk, chain_only=bool(chain))
    _log(f"eigen {name}: power iteration to {tol:g} ...")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi, k, st = s.solve_eigen(nsf, chi, tol=tol, max_iters=max_iters)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    segg = st["seg_group_updates"]
    out = {"study": "eigen", "workload": name, "tol": tol, "k_eff": k, "iterations": st["iters"],
           "converged": st["converged"], "residual": st["residual"], "wall_s": wall,
           "ms_per_iteration": wall / st["iters"] * 1e3, "sweep_ms_median": st["sweep_ms_median"],
           "seg_group_updates_per_sweep": segg,
           "seg_group_per_s_wall": segg * st["iters"] / wall, "walk": s.walk(), "chain": bool(chain)}
    s.close()
    return out


SCHEDULES = [
    # label, (order, persistent), store fraction of free device memory
    ("otf longest-first (default)", ("longest_first", False), None),
    ("otf natural order", ("natural", False), None),
    ("otf natural, persistent grid", ("natural", True), None),
    ("otf decreasing work, persistent grid", ("longest_first", True), None),
    ("otf alternating groups, persistent grid", ("alternating", True), None),
    ("exp longest-first", ("longest_first", False), 0.8),
    ("exp alternating groups, persistent grid", ("alternating", True), 0.8),
]


def exp_study(name, iters=10, labels=None):
    """Stored-segment (EXP) sweep and work-unit schedules (paper sections 4.2
    and 4.3): median sweep time of each variant over `iters` iterations, the
    store's share of the walk's steps and its setup time."""
    import torch
    prob = P.get(name)
    plan = moc.Plan(prob)
    out = {"study": "exp", "workload": name, "iterations": iters, "variants": []}
    for label, sched, store in SCHEDULES:
        if labels and label not in labels:
            continue
        s = moc.Solver(plan, fp64_boundary=False)
        s.set_source(prob.q)
        s.set_schedule(*sched)
        info, t_store = None, 0.0
        if store:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = s.store_segments(fraction=store)
            torch.cuda.synchronize()
            t_store = time.perf_counter() - t0
        s.reset()
        s.iterate(2, stats=False)
        st = s.iterate(iters)
        row = {"variant": label, "sweep_ms_median": st["sweep_ms_median"],
               "seg_group_per_s": st["seg_group_updates"] / (st["sweep_ms_median"] * 1e-3)}
        if info:
            row.update(store_s=t_store, units_stored=info["units_stored"],
                       units_total=info["units_total"], store_gb=info["bytes_used"] / 1e9,
                       steps_stored_frac=info["wave_steps_stored"] / max(info["wave_steps_total"], 1))
        _log(f"exp {name}: {row}")
        out["variants"].append(row)
        s.close()
        del s
        torch.cuda.empty_cache()
    return out


def window_study(name, iters=5, sizes=(256, 512, 1024)):
    """Median sweep time of the per-lane sweep for each workgroup size whose
    window fits (threads, 2D segments per window)."""
    import torch
    prob = P.get(name)
    plan = moc.Plan(prob)
    out = {"study": "window", "workload": name, "iterations": iters, "sizes": []}
    s = moc.Solver(plan, fp64_boundary=False)
    s.set_source(prob.q)
    out["automatic"] = s.window()
    for nt in sizes:
        try:
            s.set_window(nt)
        except moc.MocError:
            continue
        s.reset()
        s.iterate(1, stats=False)
        st = s.iterate(iters)
        row = {"threads": nt, "segments_per_window": s.window()[1],
               "sweep_ms_median": st["sweep_ms_median"],
               "seg_group_per_s": st["seg_group_updates"] / (st["sweep_ms_median"] * 1e-3)}
        _log(f"window {name}: {row}")
        out["sizes"].append(row)
    s.close()
    return out


def bundles_study(name, iters=5, sizes=(256, 512, 1024), rounds=2):
    """Median sweep time with static and with dynamic bundle assignment, for
    each workgroup size whose window fits, in interleaved rounds."""
    prob = P.get(name)
    plan = moc.Plan(prob)
    out = {"study": "bundles", "workload": name, "iterations": iters, "rows": []}
    s = moc.Solver(plan, fp64_boundary=False)
    s.set_source(prob.q)
    out["automatic"] = s.window()
    for nt in sizes:
        try:
            s.set_window(nt)
        except moc.MocError:
            continue
        for r in range(rounds):
            for mode in ("static", "dynamic"):
                s.set_bundles(mode)
                s.reset()
                s.iterate(1, stats=False)
                st = s.iterate(iters)
                row = {"threads": nt, "segments_per_window": s.window()[1], "bundles": mode,
                       "round": r, "sweep_ms_median": st["sweep_ms_median"],
                       "seg_group_per_s": st["seg_group_updates"] / (st["sweep_ms_median"] * 1e-3)}
                _log(f"bundles {name}: {row}")
                out["rows"].append(row)
    s.set_bundles("auto")
    s.close()
    return out


def chain_study(name, iters=5, tol=1e-6, max_iters=2000, sizes=(0,)):
    """Lagged boundary flux against chain-line sweeping: median sweep time
    over `iters` iterations of each (per workgroup size in `sizes`, 0 the
    automatic one), then, with tol > 0, the source iterations and wall time
    each needs to reach tol."""
    import torch
    prob = P.get(name)
    plan = moc.Plan(prob)
    out = {"study": "chain", "workload": name, "iterations": iters, "tol": tol, "rows": []}
    s = moc.Solver(plan, fp64_boundary=False)
    s.set_source(prob.q)
    for nt in sizes:
        s.set_window(nt)
        for chain in (0, 1):
            s.set_chain(chain)
            s.reset()
            s.iterate(1, stats=False)
            st = s.iterate(iters)
            row = {"mode": ("lagged", "chain")[chain], "threads": s.window()[0],
                   "segments_per_window": s.window()[1], "sweep_ms_median": st["sweep_ms_median"],
                   "seg_group_per_s": st["seg_group_updates"] / (st["sweep_ms_median"] * 1e-3)}
            _log(f"chain {name}: {row}")
            out["rows"].append(row)
    s.set_window(0)
    if tol > 0:
        out["converge"] = []
        for chain in (0, 1):
            s.set_chain(chain)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            phi, st = s.solve(tol=tol, max_iters=max_iters)
            torch.cuda.synchronize()
            row = {"mode": "chain" if chain else "lagged", "iters": st["iters"],
                   "converged": st["converged"], "residual": st["residual"],
                   "wall_s": time.perf_counter() - t0, "sweep_ms_median": st["sweep_ms_median"]}
            _log(f"chain {name} converge: {row}")
            out["converge"].append(row)
        s.set_chain(0)
    s.close()
    return out


def chain_only_study(name, iters=10):
    """A chain-only solver (workspace without boundary buffers): workspace
    size against the full one, median sweep time and residual history over
    `iters` source iterations."""
    import torch
    prob = P.get(name)
    plan = moc.Plan(prob)
    info = plan.info
    s = moc.Solver(plan, chain_only=True)
    s.set_source(prob.q)
    hist, sweeps = [], []
    t0 = time.perf_counter()
    for k in range(iters):
        st = s.iterate(1)
        hist.append(st["residual"])
        sweeps.append(st["sweep_ms_median"])
        _log(f"chain-only {name}: iteration {k + 1}/{iters} residual {st['residual']:.3e} "
             f"sweep {st['sweep_ms_median']:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"study": "chain_only", "workload": name, "iterations": iters,
           "workspace_bytes_full": info["workspace_bytes"],
           "workspace_bytes_chain": info["workspace_bytes_chain"],
           "allocated_bytes": int(s.workspace.numel()), "wall_s": wall,
           "sweep_ms_median": float(np.median(sweeps)),
           "seg_group_per_s": st["seg_group_updates"] / (float(np.median(sweeps)) * 1e-3),
           "residual_history": hist, "seg_group_updates_per_sweep": st["seg_group_updates"],
           "link_errors": st["link_errors"], "window": s.window(),
           "segments": info["n_chain_segments"]}
    s.close()
    return out


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=("precision", "scale", "eigen", "exp", "window", "bundles", "chain",
                                     "chain_only"))
    ap.add_argument("--workload", default=None)
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--walk", choices=("auto", "lockstep", "lane"), default="auto")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--chain", action="store_true", help="eigen: chain-line sweeps (chain-only solver)")
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if args.study == "precision":
        out = precision(args.workload or "lattice32", args.iters or 20)
    elif args.study == "window":
        out = window_study(args.workload or "lattice32", args.iters or 5)
    elif args.study == "bundles":
        out = bundles_study(args.workload or "lattice32", args.iters or 5)
    elif args.study == "exp":
        out = exp_study(args.workload or "lattice8", args.iters or 10)
    elif args.study == "chain_only":
        out = chain_only_study(args.workload or "lattice64", args.iters or 10)
    elif args.study == "chain":
        out = chain_study(args.workload or "lattice8", args.iters or 5, tol=args.tol)
    elif args.study == "eigen":
        out = eigen(args.workload or "lattice8", max_iters=args.iters or 2000, chain=args.chain)
    else:
        out = scale(args.workload or "lattice64", args.iters or 50, args.walk)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
