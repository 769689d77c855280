"""Benchmark: segment-group integrations per second of fixed-source 3D MOC
source iterations on one MI355X.

A step is one source iteration over the whole problem: source update, the
on-the-fly 3D sweep (segment generation, Eq. 3 attenuation, FSR tally,
boundary flux exchange) and the finalize pass.  Inputs are resident in HBM
before the timed region.  Prints one JSON line.

The headline workload is the largest single-GPU lattice (lattice64: 64x64
pin cells, 200 layers, 7 groups, 64 x 8 angles, 0.03 / 0.1 cm, about 7.2e12
segment-group updates per sweep).  The oracle cannot run whole iterations
there, so the CPU leg sweeps a seeded sample of directed tracks once, in FP64,
from the GPU's own reduced source and boundary flux after the timed
iterations: that sample gives the parity figures (outgoing flux per track and
FSR tallies) and the oracle's rate.  The small lattice8 problem also runs in
full beside it, with 56 whole oracle iterations for parity.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lattice64]
"""
import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_SEG_GROUP = 12.0      # 4 B reduced-source gather + 8 B FP64 tally update
# Vector ALU issue peak: 256 CUs x 4 SIMDs, each retiring one wave64 VALU
# issue slot every 4 cycles (16 lanes per cycle), at 2.4 GHz; an ordinary
# instruction takes one slot, a transcendental two
VALU_PEAK_INSTR_PER_S = 256 * 4 * 2.4e9 / 4


def workload_desc(prob):
    return (f"{prob.name}: {prob.nx}x{prob.ny} pin cells (pitch {prob.pitch} cm, inclusion "
            f"r={prob.radius} cm, {prob.n_sectors} sectors x 2 rings), {prob.height:g} cm in "
            f"{prob.n_layers} layers, {prob.n_groups} groups, {prob.n_azim} azimuthal x "
            f"{prob.n_polar} polar, {prob.radial_spacing}/{prob.axial_spacing} cm spacing")


def kernel_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2503_17743_amd", "csrc", "sweep.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def load_counters(workload):
    """The sweep kernel's rocprofv3 counter summary for this workload
    (profiles/counters_<workload>.json), or None when absent or taken on a
    different sweep source."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_hash") != kernel_hash():
        return None
    return rec


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def oracle_threads():
    return max(1, min(16, len(os.sched_getaffinity(0))))


# ------------------------------------------------------------------ CPU leg
def full_oracle(prob, iters, threads):
    """The oracle's whole-problem iterations (small workloads)."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    m = O.Model(prob, n_threads=threads)
    t1 = time.perf_counter()
    phi, _ = m.solve(max_iters=iters, tol=0.0)
    t2 = time.perf_counter()
    seg_groups = 2 * m.info["n_segments"] * prob.n_groups * iters
    return phi, {
        "value": seg_groups / (t2 - t1),
        "unit": "seg-group/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{iters} FP64 source iterations of the full {prob.name} problem "
                   f"(trace/setup {t1 - t0:.1f} s excluded, sweep+update {t2 - t1:.1f} s)"),
    }


def sampled_parity(prob, plan, solver, n_tracks, seed, threads):
    """One sweep of a seeded sample of whole work items (bundles of
    consecutive lines of one z-stack, one direction; at least n_tracks
    directed tracks) on the GPU and in the FP64 oracle, from the same inputs:
    the reduced source of the solver's last iteration and the boundary flux
    its next sweep reads (zero where a track enters through a vacuum face, as
    the oracle decides).  The GPU sweep runs the kernel of the timed path
    restricted to the sample.

    Compared: every track's outgoing angular flux, and every FSR-group tally
    of the sample, relatively but with a floor: the flat-source term
    qhat Sigma_t sum W l of the same sampled path (path lengths sum W l per FSR
    from the oracle).  A tally sums W (psi - qhat) F(tau), whose terms change
    sign; where psi and qhat nearly cancel, only its error against that
    floor is meaningful.  Also reported: the FSR flux the sample's own tracks
    estimate (Eq. 4 over the sampled segments), whose relative error is
    large only where that estimate itself is near zero (psi near 0 on a
    short path).  Returns the comparison and the oracle's timing; the
    solver's iterate is consumed (the hook resets it)."""
    import numpy as np
    from oracle import oracle as O
    G, T = prob.n_groups, plan.info["tracks_per_wave"]
    rng = np.random.default_rng(seed)
    n_cand = min(2 * plan.info["n_chunks"], int(np.ceil(1.25 * n_tracks / T)) + 8)
    cand = rng.choice(2 * plan.info["n_chunks"], size=n_cand, replace=False)
    chosen, total = [], 0
    for it in cand:
        if total >= n_tracks:
            break
        chosen.append(int(it))
        total += plan.chunk(int(it) // 2)[1]
    items = np.sort(np.array(chosen, np.int64))
    n_items = len(items)
    tracks, dirs, rows = [], [], []
    for i, it in enumerate(items):
        ft, nt = plan.chunk(int(it) // 2)
        for k in range(nt):
            tracks.append(ft + k)
            dirs.append(int(it) % 2)
            rows.append((i, k))
    tracks = np.array(tracks, np.int64)
    dirs = np.array(dirs, np.int32)
    qhat = solver.reduced_source()
    psi = solver.boundary_flux(2 * tracks + dirs)
    om = O.Model(prob, trace=False)
    psi[om.entry_vacuum(tracks, dirs)] = 0.0
    psi_items = np.zeros((n_items, T, G))
    for (i, k), v in zip(rows, psi):
        psi_items[i, k] = v
    acc_g, psi_out_g = solver.sweep_items(items, qhat, psi_items)
    gpsi = np.array([psi_out_g[i, k] for i, k in rows])
    # oracle: the sample split over threads (ctypes releases the GIL), each
    # with its own tally array, summed afterwards
    parts = np.array_split(np.arange(len(tracks)), threads)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda ix: om.sweep_sample(tracks[ix], dirs[ix], qhat, psi[ix]), parts))
    wall = time.perf_counter() - t0
    opsi = np.concatenate([r[1] for r in res])
    nseg = int(sum(r[2] for r in res))
    acc_o = res[0][0]
    for r in res[1:]:
        acc_o += r[0]
    del res
    with cf.ThreadPoolExecutor(threads) as ex:
        wls = list(ex.map(lambda ix: om.sample_path_length(tracks[ix]), parts))
    wl = wls[0]
    for w in wls[1:]:
        wl += w
    del wls

    four_pi = 4.0 * np.pi
    rel_psi = np.abs(gpsi - opsi) / np.maximum(np.abs(opsi), 1e-300)
    touched = wl > 0
    st = prob.sigma_t[prob.fsr_material()[touched]]          # [n_touched][G]
    denom = st * wl[touched][:, None]
    # tallies: relative error with a per-FSR-group floor, the flat-source term
    # qhat Sigma_t sum W l of the same sampled path (where psi and qhat nearly
    # cancel, the tally is small and only its absolute error means anything)
    floor = qhat[touched] * denom
    dacc = np.abs(acc_g[touched] - acc_o[touched])
    rel_acc = dacc / np.maximum(np.maximum(np.abs(acc_o[touched]), floor), 1e-300)
    # the FSR flux the sampled tracks alone estimate (Eq. 4 over the sample)
    phi_o = four_pi * qhat[touched] + four_pi * acc_o[touched] / denom
    phi_g = four_pi * qhat[touched] + four_pi * acc_g[touched] / denom
    rel_phi = np.abs(phi_g - phi_o) / np.maximum(np.abs(phi_o), 1e-300)
    out = {
        "tracks": int(len(tracks)),
        "segments": nseg,
        "max_rel_err_psi_out": float(rel_psi.max()),
        "fsr_groups_touched": int(touched.sum()) * G,
        "max_rel_err_tally": float(rel_acc.max()),
        "tally_floor": "qhat * Sigma_t * sum(W l) of the sampled path, per FSR-group",
        "sample_fsr_flux_rel_err_p999": float(np.percentile(rel_phi, 99.9)),
        "sample_fsr_flux_rel_err_max": float(rel_phi.max()),
        "tallies_outside_sample": int((np.abs(acc_g[~touched]) > 0).sum()),
    }
    cpu = {
        "value": nseg * G / wall,
        "unit": "seg-group/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{len(tracks)} seeded directed tracks of {prob.name} ({nseg} segments) traced "
                   f"by brute force and swept once in FP64 in {wall:.2f} s on {threads} threads; "
                   f"rate extrapolated to the whole sweep"),
        "extrapolated": True,
    }
    return out, cpu, (gpsi, opsi, phi_g, phi_o)


# ------------------------------------------------------------------ GPU legs
def timed_iterations(solver, steps, warmup, name=""):
    """Warm-up, then exactly `steps` timed iterations.  Long iterations are
    issued in chunks of about 20 s, each ending in a progress line (the
    chunk's own stats read synchronises once); short ones in one call."""
    import torch
    solver.reset()
    torch.cuda.synchronize()
    per_step = 0.0
    for k in range(warmup):
        t0 = time.perf_counter()
        solver.iterate(1, stats=False)
        torch.cuda.synchronize()
        per_step = time.perf_counter() - t0
        if per_step > 1.0:
            log(f"{name}: warm-up iteration {k + 1}/{warmup} ({per_step:.1f} s)")
    chunk = steps if per_step < 1.0 else max(1, int(20.0 / per_step))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, st = 0, None
    while done < steps:
        n = min(chunk, steps - done)
        st = solver.iterate(n, stats=True)
        done += n
        if chunk < steps:
            log(f"{name}: timed iteration {done}/{steps} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return st, time.perf_counter() - t0


def small_workload(name, steps, oracle_iters, cpu_leg):
    """Whole-problem line of a small workload, with full-oracle parity."""
    import numpy as np
    from paper_2503_17743_amd import moc, problems as P
    prob = P.get(name)
    plan = moc.Plan(prob)
    solver = moc.Solver(plan, fp64_boundary=False, chain_only=False)
    solver.set_source(prob.q)
    parity, cpu = None, None
    if cpu_leg:
        log(f"{name}: {oracle_iters} oracle iterations ...")
        ophi, cpu = full_oracle(prob, oracle_iters, oracle_threads())
        solver.reset()
        solver.iterate(oracle_iters, stats=False)
        gphi = solver.flux()
        parity = float(np.max(np.abs(gphi - ophi) / np.maximum(np.abs(ophi), 1e-300)))
    log(f"{name}: timed iterations ...")
    st, elapsed = timed_iterations(solver, steps, 3, name)
    solver.close()
    segg = st["seg_group_updates"]
    return {
        "workload": workload_desc(prob),
        "value": segg * steps / elapsed,
        "steps": steps,
        "ms_per_step": elapsed / steps * 1e3,
        "sweep_ms_median": st["sweep_ms_median"],
        "seg_group_updates_per_step": segg,
        "max_rel_err_vs_fp64_oracle": parity,
        "parity_iterations": oracle_iters if parity is not None else None,
        "cpu_baseline": cpu,
    }


def chain_leg(name, iters, cpu_leg):
    """Chain-line sweeping on a small workload: a chain-only solver (no
    boundary buffers) against the full lagged one, its sweep time, and its
    iterate after `iters` iterations against the oracle's chain iterate."""
    import numpy as np
    from paper_2503_17743_amd import moc, problems as P
    prob = P.get(name)
    plan = moc.Plan(prob)
    solver = moc.Solver(plan, chain_only=True)
    solver.set_source(prob.q)
    log(f"{name}: {iters} chain-line iterations ...")
    st = solver.iterate(iters)
    gphi = solver.flux()
    window = solver.window()
    solver.close()
    parity = None
    if cpu_leg:
        from oracle import oracle as O
        m = O.Model(prob, n_threads=oracle_threads())
        ophi, _ = m.solve(max_iters=iters, tol=0.0, chain=True)
        parity = float(np.max(np.abs(gphi - ophi) / np.maximum(np.abs(ophi), 1e-300)))
    return {
        "workload": name,
        "iterations": iters,
        "sweep_ms_median": st["sweep_ms_median"],
        "seg_group_per_s": st["seg_group_updates"] / (st["sweep_ms_median"] * 1e-3),
        "workspace_bytes_chain_only": plan.info["workspace_bytes_chain"],
        "workspace_bytes_lagged": plan.info["workspace_bytes"],
        "link_errors": st["link_errors"],
        "threads": window[0],
        "max_rel_err_vs_fp64_oracle_chain": parity,
    }


def chain_headline(prob, plan, steps, segg_lagged):
    """Chain-line sweeps of the headline workload in a chain-only solver (no
    boundary buffers): median sweep time, the same segment-group count as
    the lagged sweep, and the two workspace sizes."""
    from paper_2503_17743_amd import moc
    solver = moc.Solver(plan, chain_only=True)
    solver.set_source(prob.q)
    log(f"{prob.name}: 1 + {steps} chain-line iterations (chain-only solver) ...")
    solver.iterate(1, stats=False)
    st = solver.iterate(steps)
    solver.close()
    return {
        "iterations": steps,
        "sweep_ms_median": st["sweep_ms_median"],
        "seg_group_per_s": st["seg_group_updates"] / (st["sweep_ms_median"] * 1e-3),
        "seg_group_updates_equal_lagged": st["seg_group_updates"] == segg_lagged,
        "link_errors": st["link_errors"],
        "workspace_bytes_chain_only": plan.info["workspace_bytes_chain"],
        "workspace_bytes_lagged": plan.info["workspace_bytes"],
        "segments": plan.info["n_chain_segments"],
    }


def roofline(segg, sweep_s, counters):
    """The sweep's binding roof: vector ALU issue (measured wave64 VALU issue
    slots per launch, SQ_ACTIVE_INST_VALU, in which a transcendental counts
    twice, over the kernel time), with the instruction count, the algorithmic
    HBM figure and the measured DRAM traffic as context."""
    eff_gbs = BYTES_PER_SEG_GROUP * segg / sweep_s / 1e9
    line = {"bound": "alu", "achieved": None, "peak": VALU_PEAK_INSTR_PER_S,
            "unit": "wave64 VALU issue slots/s", "frac": None, "traffic": None,
            "effective_hbm_gbs": eff_gbs, "effective_hbm_frac": eff_gbs / HBM_PEAK_GBS}
    if counters is not None:
        valu = counters["valu_instructions_per_launch"]
        slots = counters.get("valu_issue_slots_per_launch", valu)
        line["achieved"] = slots / sweep_s
        line["frac"] = line["achieved"] / VALU_PEAK_INSTR_PER_S
        line["valu_instructions_per_s"] = valu / sweep_s
        line["valu_instructions_frac"] = valu / sweep_s / VALU_PEAK_INSTR_PER_S
        line["traffic"] = counters.get("hbm_bytes_per_launch")
        if line["traffic"]:
            line["dram_gbs"] = line["traffic"] / sweep_s / 1e9
        line["counters"] = dict(counters.get("limiters", {}), source=counters.get("source"),
                                kernel=counters.get("kernel"))
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="lattice64")
    ap.add_argument("--small-workload", default="lattice8",
                    help="a small problem also run in full, with whole-oracle parity ('' to skip)")
    ap.add_argument("--small-steps", type=int, default=30)
    ap.add_argument("--oracle-iters", type=int, default=56,
                    help="whole oracle iterations of the small workload")
    ap.add_argument("--sample-tracks", type=int, default=400000,
                    help="directed tracks of the sampled oracle sweep on the headline workload")
    ap.add_argument("--walk", choices=("auto", "lockstep", "lane"), default="auto")
    ap.add_argument("--chain-workload", default="lattice8",
                    help="a small problem also swept in chain-line mode ('' to skip)")
    ap.add_argument("--chain-iters", type=int, default=5)
    ap.add_argument("--chain-steps", type=int, default=2,
                    help="chain-line sweeps of the headline workload in a chain-only solver (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=32,
                    help="requests in the serving comparison (0: skip it)")
    ap.add_argument("--serving-arena-gib", type=float, default=8.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the sweep runs on a single GPU "
              "(the multi-GPU angular decomposition is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2503_17743_amd import moc, problems as P, serve as S

    torch.cuda.set_device(0)
    if args.copy_calibration:
        # a plain copy of known size: reads 1 GiB and writes 1 GiB of HBM
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    small = None
    if args.small_workload:
        small = small_workload(args.small_workload, args.small_steps, args.oracle_iters,
                               not args.no_cpu_baseline)
    chain = None
    if args.chain_workload:
        chain = chain_leg(args.chain_workload, args.chain_iters, not args.no_cpu_baseline)
    serving = None
    if args.serving_requests > 0:
        serving = S.compare(args.serving_requests, args.serving_arena_gib, log=log)
        # smaller requests (coarser tracking): per-iteration overheads matter more
        serving["small_requests"] = S.compare(2 * args.serving_requests, args.serving_arena_gib,
                                              radial=0.2, axial=0.5, poisson=False, log=log)
    torch.cuda.empty_cache()

    prob = P.get(args.workload)
    t0 = time.perf_counter()
    plan = moc.Plan(prob)
    log(f"{prob.name}: planned in {time.perf_counter() - t0:.1f} s, workspace "
        f"{plan.info['workspace_bytes'] / 1e9:.1f} GB")
    solver = moc.Solver(plan, fp64_boundary=False, walk=args.walk, chain_only=False)
    solver.set_source(prob.q)
    log(f"{prob.name}: {args.warmup} warm-up + {args.steps} timed iterations ...")
    st, elapsed = timed_iterations(solver, args.steps, args.warmup, prob.name)
    segg = st["seg_group_updates"]
    value = segg * args.steps / elapsed
    sweep_s = st["sweep_ms_median"] * 1e-3
    balance_rel = abs(st["balance_lhs"] - st["balance_rhs"]) / max(abs(st["balance_rhs"]), 1e-300)
    log(f"{prob.name}: {value:.3e} seg-group/s, sweep {st['sweep_ms_median']:.1f} ms, "
        f"residual {st['residual']:.2e}")
    parity, cpu = None, None
    if not args.no_cpu_baseline:
        log(f"{prob.name}: sampled oracle sweep of {args.sample_tracks} tracks ...")
        parity, cpu, _ = sampled_parity(prob, plan, solver, args.sample_tracks, seed=17,
                                        threads=oracle_threads())
        log(f"{prob.name}: parity {parity}")
    solver_walk = solver.walk()
    solver.close()
    torch.cuda.empty_cache()
    chain_head = None
    if args.chain_steps > 0 and plan.info["workspace_bytes_chain"]:
        chain_head = chain_headline(prob, plan, args.chain_steps, segg)
        log(f"{prob.name}: chain-line sweep {chain_head['sweep_ms_median']:.1f} ms")

    line = {
        "metric": "segment-group integrations/s at 1e-5 vs FP64",
        "value": value,
        "unit": "seg-group/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": workload_desc(prob),
            "seg_group_updates_per_step": segg,
            "n_fsr": plan.info["n_fsr"],
            "n_3d_tracks": plan.info["n_3d_tracks"],
            "workspace_bytes": plan.info["workspace_bytes"],
            "accumulation": "f64",
            "sweep_ms_median": st["sweep_ms_median"],
            "residual_last_step": st["residual"],
            "balance_rel_last_step": balance_rel,
            "link_errors": st["link_errors"],
            "walk": solver_walk,
            "sampled_oracle_parity": parity,
            "small_workload": small,
            "chain_line": chain,
            "chain_line_headline": chain_head,
        },
        "roofline": roofline(segg, sweep_s, load_counters(prob.name)),
        "cpu_baseline": cpu,
        "serving": serving,
        # the paper's own figures, for context only (other hardware, C5G7 3D
        # eigenvalue benchmark, no absolute times survive in its text)
        "paper_context": ("GPU OTF 30x rising to about 100x over OpenMOC's CPU OTF as the problem "
                          "grows (section 5.2), on GTX 1080Ti / RTX 2080Ti / RTX 3060 / RTX 4090 "
                          "with an i7-12700KF, and an MI60 with a 32-core CPU (Table 1)"),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
