"""Serving driver: a stream of independent fixed-source requests, run through
the continuous-batching server and, for comparison, one at a time in arrival
order on the same GPU.  Latency of a request = its completion time minus its
arrival time; throughput = requests (and segment-group updates) per second of
wall time."""
from __future__ import annotations

import sys
import time
from typing import Dict, List

import numpy as np

from . import moc, problems as P


def _stderr(msg):
    print(msg, file=sys.stderr, flush=True)


def plan_requests(reqs: List[P.Request]):
    return [moc.Plan(r.problem) for r in reqs]


def _arrivals(reqs, use_arrivals):
    return np.array([r.arrival_s for r in reqs]) if use_arrivals else np.zeros(len(reqs))


def _progress(log, every, k, n, what):
    if log is not None and every and (k % every == 0 or k == n):
        log(f"{what}: {k}/{n} requests done")


def one_at_a_time(reqs, plans, tol, max_iters, use_arrivals=False, log=None, log_every=0,
                  stream="own"):
    """FIFO, one request on the GPU at a time: wait for its arrival, bind a
    solver, solve to tol, read the flux back, release the workspace.
    stream="own": each solve on a stream of its own, every iteration one
    captured graph; "current": plain launches on torch's current stream.
    `log(msg)` is called every `log_every` completed requests (0: never)."""
    import torch
    arr = _arrivals(reqs, use_arrivals)
    out, stats = [], []
    lat = np.zeros(len(reqs))
    segg = 0
    t0 = time.perf_counter()
    for i, (r, pl) in enumerate(zip(reqs, plans)):
        wait = arr[i] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        s = moc.Solver(pl, fp64_boundary=False, stream=stream)
        s.set_source(r.problem.q)
        phi, st = s.solve(tol=tol, max_iters=max_iters)
        s.close()
        del s
        lat[i] = time.perf_counter() - t0 - arr[i]
        segg += st["seg_group_updates"] * st["iters"]
        out.append(phi)
        stats.append(st)
        _progress(log, log_every, i + 1, len(reqs), "one at a time")
    torch.cuda.synchronize()
    return out, {"wall_s": time.perf_counter() - t0, "seg_group_updates": segg,
                 "latency_s": lat.tolist(), "stats": stats}


def run_stream(reqs, plans, tol, max_iters, arena_bytes, max_slots=64, use_arrivals=False,
               fill_units=None, log=None, log_every=0, classes=1, split_units=None):
    """Submit each request at its arrival time (all at t=0 unless use_arrivals)
    and step the server until every request is done (progress as for
    one_at_a_time).  classes=2: requests below split_units work units (default:
    1/16 of the fill target) go to a second server with its own stream and a
    quarter of the arena, so small requests step at their own rate while the
    large ones' kernels run beside them."""
    n = len(reqs)
    if classes == 2:
        small_bytes = arena_bytes // 4
        srvs = [moc.Server(arena_bytes - small_bytes, max_slots=max_slots, fill_units=fill_units),
                moc.Server(small_bytes, max_slots=max_slots, fill_units=fill_units)]
        if split_units is None:
            import torch
            cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
            split_units = (fill_units or 64 * cus) // 16
        route = [1 if 2 * pl.info["n_2d_tracks"] < split_units else 0 for pl in plans]
    else:
        srvs = [moc.Server(arena_bytes, max_slots=max_slots, fill_units=fill_units)]
        route = [0] * n
    arr = _arrivals(reqs, use_arrivals)
    tickets: Dict[tuple, int] = {}
    done: Dict[int, tuple] = {}
    lat = np.zeros(n)
    segg = 0
    steps = 0
    max_active = 0
    t0 = time.perf_counter()
    nxt = 0
    while len(done) < n:
        now = time.perf_counter() - t0
        while nxt < n and arr[nxt] <= now:
            k = route[nxt]
            tickets[(k, srvs[k].submit(plans[nxt], reqs[nxt].problem.q, tol, max_iters))] = nxt
            nxt += 1
        if not tickets:
            time.sleep(max(0.0, min(arr[nxt] - now, 0.01)))
            continue
        na = 0
        for k, srv in enumerate(srvs):
            if any(kk == k for kk, _ in tickets):
                a, _ = srv.step()
                na += a
        steps += 1
        max_active = max(max_active, na)
        now = time.perf_counter() - t0
        for key in list(tickets):
            res = srvs[key[0]].poll(key[1])
            if res is None:
                continue
            i = tickets.pop(key)
            done[i] = res
            lat[i] = now - arr[i]
            segg += res[1]["seg_group_updates"] * res[1]["iters"]
            _progress(log, log_every, len(done), n, "batched")
    wall = time.perf_counter() - t0
    for srv in srvs:
        srv.close()
    return [done[i][0] for i in range(n)], {
        "wall_s": wall, "seg_group_updates": segg, "latency_s": lat.tolist(), "steps": steps,
        "max_active": max_active, "stats": [done[i][1] for i in range(n)]}


def summarize(d, n):
    lat = np.array(d["latency_s"])
    out = {"requests": n, "wall_s": d["wall_s"], "req_per_s": n / d["wall_s"],
           "seg_group_per_s": d["seg_group_updates"] / d["wall_s"],
           "latency_p50_s": float(np.percentile(lat, 50)),
           "latency_p99_s": float(np.percentile(lat, 99))}
    if "max_active" in d:
        out["max_active"] = d["max_active"]
    return out


def max_rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def _pool(runs, n):
    """Summary of repeated runs of one mode: mean wall time, pooled latencies."""
    wall = float(np.mean([d["wall_s"] for d in runs]))
    lat = np.concatenate([np.array(d["latency_s"]) for d in runs])
    out = {"requests": n, "runs": len(runs), "wall_s": wall, "wall_s_each": [d["wall_s"] for d in runs],
           "req_per_s": n / wall,
           "seg_group_per_s": float(np.mean([d["seg_group_updates"] / d["wall_s"] for d in runs])),
           "latency_p50_s": float(np.percentile(lat, 50)),
           "latency_p99_s": float(np.percentile(lat, 99))}
    if "max_active" in runs[0]:
        out["max_active"] = max(d["max_active"] for d in runs)
    return out


def compare(n_requests, arena_gib, tol=1e-6, max_iters=400, load=0.8, radial=0.05,
            axial=0.2, poisson=True, log=None, log_every=0, repeats=2, two_class=True):
    """Continuous batching against one-at-a-time on the same seeded requests:
    first all arriving at once (throughput; with repeats=2 the runs go one,
    one plain, batched, batched, one plain, one, so that no mode always runs
    on a GPU that has been busy longer; the faster one-at-a-time form is the
    baseline), then Poisson arrivals at `load` times the one-at-a-time
    service rate (latency).  Returns a JSON-ready dict."""
    def say(msg):
        if log is not None:
            log(msg)
    probs = [r.problem for r in P.serving_stream(n_requests=n_requests, radial=radial, axial=axial)]
    reqs = P.with_arrivals(probs, None)
    t0 = time.perf_counter()
    plans = plan_requests(reqs)
    tag = f"{n_requests} requests at {radial}/{axial} cm"
    say(f"serving ({tag}): planned in {time.perf_counter() - t0:.1f} s")
    arena = moc.Server.overhead_bytes(64) + int(arena_gib * (1 << 30))
    kw = dict(log=log, log_every=log_every)
    # one at a time in both launch forms (graph-captured iterations on an own
    # stream, plain launches); the faster is the baseline of the ratio
    order = (("one", "one_plain", "batched", "batched", "one_plain", "one") if repeats >= 2
             else ("one", "one_plain", "batched"))
    runs = {"one": [], "one_plain": [], "batched": []}
    phi = {}
    for mode in order:
        say(f"serving ({tag}): {mode} ...")
        if mode == "one":
            phi[mode], d = one_at_a_time(reqs, plans, tol, max_iters, **kw)
        elif mode == "one_plain":
            phi[mode], d = one_at_a_time(reqs, plans, tol, max_iters, stream="current", **kw)
        else:
            phi[mode], d = run_stream(reqs, plans, tol, max_iters, arena, **kw)
        runs[mode].append(d)
        say(f"serving ({tag}): {mode} {d['wall_s']:.2f} s")
    err = max(max_rel(a, b) for a, b in zip(phi["batched"], phi["one"]))
    conv = all(st["converged"] for d in runs["batched"] + runs["one"] + runs["one_plain"]
               for st in d["stats"])
    one_g, one_p = _pool(runs["one"], n_requests), _pool(runs["one_plain"], n_requests)
    bat = _pool(runs["batched"], n_requests)
    one = one_g if one_g["wall_s"] <= one_p["wall_s"] else one_p
    out = {
        "workload": (f"{n_requests} independent fixed-source lattice solves to residual {tol:g} "
                     f"(4x4/8x8/16x16 cells, 10-50 layers, 1-7 groups, 8-32 azimuthal x 2-6 "
                     f"polar, {radial}/{axial} cm spacing)"),
        "arena_bytes": arena,
        "all_converged": conv,
        "max_rel_diff_batched_vs_alone": err,
        "offline": {"order": list(order), "batched": bat, "one_at_a_time_graphs": one_g,
                    "one_at_a_time_plain": one_p,
                    "baseline": "graphs" if one is one_g else "plain",
                    "throughput_ratio": one["wall_s"] / bat["wall_s"],
                    "throughput_ratio_each_run": [o["wall_s"] / b["wall_s"] for o, b in
                                                  zip(runs["one" if one is one_g else "one_plain"],
                                                      runs["batched"])]},
    }
    if two_class:
        say(f"serving ({tag}): batched, two classes ...")
        _, b2 = run_stream(reqs, plans, tol, max_iters, arena, classes=2, **kw)
        say(f"serving ({tag}): batched, two classes {b2['wall_s']:.2f} s")
        out["offline"]["batched_two_class"] = summarize(b2, n_requests)
        out["offline"]["throughput_ratio_two_class"] = one["wall_s"] / b2["wall_s"]
    if poisson:
        rate = load * n_requests / one["wall_s"]
        preqs = P.with_arrivals(probs, rate)
        say(f"serving ({tag}): Poisson arrivals at {rate:.1f}/s, one at a time ...")
        _, pseq = one_at_a_time(preqs, plans, tol, max_iters, use_arrivals=True,
                                stream="own" if one is one_g else "current", **kw)
        say(f"serving ({tag}): Poisson one at a time {pseq['wall_s']:.2f} s; batched ...")
        _, pbat = run_stream(preqs, plans, tol, max_iters, arena, use_arrivals=True, **kw)
        say(f"serving ({tag}): Poisson batched {pbat['wall_s']:.2f} s")
        out["poisson"] = {"rate_req_per_s": rate, "load": load,
                          "batched": summarize(pbat, n_requests),
                          "one_at_a_time": summarize(pseq, n_requests)}
        if two_class:
            _, p2 = run_stream(preqs, plans, tol, max_iters, arena, use_arrivals=True, classes=2, **kw)
            say(f"serving ({tag}): Poisson batched, two classes {p2['wall_s']:.2f} s")
            out["poisson"]["batched_two_class"] = summarize(p2, n_requests)
    return out


def main(argv=None):
    """Run a seeded request stream and print one JSON summary line:
    python -m paper_2503_17743_amd.serve [--requests N] [--mode batched|one|compare]
    `compare` runs both ways, all at t=0 and then under Poisson arrivals at
    --load times the one-at-a-time rate; progress goes to stderr."""
    import argparse
    import json
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=32)
    ap.add_argument("--mode", choices=("batched", "one", "compare"), default="batched")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-iters", type=int, default=400)
    ap.add_argument("--arena-gib", type=float, default=8.0)
    ap.add_argument("--rate", type=float, default=0.0, help="Poisson arrivals per s (0: all at t=0)")
    ap.add_argument("--load", type=float, default=0.8, help="compare: Poisson load")
    ap.add_argument("--radial", type=float, default=0.05)
    ap.add_argument("--axial", type=float, default=0.2)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if args.mode == "compare":
        out = compare(args.requests, args.arena_gib, args.tol, args.max_iters, args.load,
                      args.radial, args.axial, log=_stderr, log_every=32)
        print(json.dumps(out), flush=True)
        return
    probs = [r.problem for r in P.serving_stream(n_requests=args.requests)]
    reqs = P.with_arrivals(probs, args.rate or None)
    plans = plan_requests(reqs)
    arrivals = args.rate > 0
    if args.mode == "one":
        _, d = one_at_a_time(reqs, plans, args.tol, args.max_iters, use_arrivals=arrivals)
    else:
        arena = moc.Server.overhead_bytes(64) + int(args.arena_gib * (1 << 30))
        _, d = run_stream(reqs, plans, args.tol, args.max_iters, arena, use_arrivals=arrivals)
    print(json.dumps({"mode": args.mode, **summarize(d, args.requests)}), flush=True)


if __name__ == "__main__":
    main()
