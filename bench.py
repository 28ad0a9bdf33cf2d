"""Throughput of the swap-MC hot path: MC swap attempts per second on one MI355X.

One step = one sweep (every site attempts one nearest-neighbour swap; Sec. V-A of the
paper): all colours (mini-steps) of trial proposal, gather, features, MLP energies, dE
reduction, Metropolis decision with FP64 re-decision near the threshold, and apply.

Default workload: BCC 256^3 cells (33,554,432 sites), 5 species equiatomic, 108-input
one-hot MLP 108 -> 128 -> 128 -> 1 (SiLU), T = 600 K, synthetic seeded inputs.

Prints one JSON line (rank 0).  --gpus N > 1 exits: this build measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_EVAL = {108: 2 * (108 * 128 + 128 * 128 + 128), 12: 2 * (12 * 64 + 64 * 64 + 64)}
OMEGA = {108: 40, 12: 22}
PEAK = {  # MI355X published dense peaks
    "fp32": (157.3e12, "mfma"), "bf16": (2.5e15, "mfma"), "bf16x3": (2.5e15, "mfma"),
    "fp8": (5.0e15, "mfma"), "fp64": (78.6e12, "mfma"),
}
DTYPE = {"fp32": "f32", "bf16": "bf16", "bf16x3": "bf16", "fp8": "fp8-e4m3", "fp64": "f64"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def run_gpu(workload, precision, steps, warmup):
    import torch

    import synth
    import paper_2604_08250_amd as smc

    w = synth.workload(workload)
    occ = w.occupancy()
    params = w.params()
    log(f"workload {workload}: {sum(w.sites):,} sites, precision {precision}")
    stream = torch.cuda.current_stream()
    mc = smc.SwapMC(w.cells, w.temperatures, occ, params, n_species=w.n_species, feature=w.feature,
                    hidden=w.hidden, precision=precision, seed=w.seed, stream=stream)
    if warmup:
        mc.sweep(warmup)
    torch.cuda.synchronize()
    mc.counters(reset=True)
    n_colours = sum(mc.n_colours(r) for r in range(mc.n_replicas))
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(steps):
        mc.sweep(1)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end)
    cnt = mc.counters()
    attempts = int(cnt[0].sum())
    diff = int(cnt[1].sum())
    accepts = int(cnt[2].sum())
    rechecks = int(cnt[3].sum())
    es, er = mc.energy()
    mc.close()
    n_sites = sum(w.sites)
    assert attempts == n_sites * steps, (attempts, n_sites, steps)
    launches = steps * n_colours
    flop = diff * OMEGA[w.n_in] * FLOP_PER_EVAL[w.n_in]
    return dict(w=w, ms=ms, wall=wall, attempts=attempts, diff=diff, accepts=accepts,
                rechecks=rechecks, launches=launches, flop=flop, e_scratch=float(es.sum()),
                e_running=float(er.sum()))


def cpu_baseline(workload, seconds=12.0):
    """The FP64 oracle, unchanged, on a bounded sample: the first trials of colour 0 of
    sweep 0 of the same workload, run on all host cores through a thread pool."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    import synth

    w = synth.workload(workload)
    cells = w.cells[0]
    occ = w.occupancy()
    model = oracle.MLP(w.feature, w.hidden, w.params())
    cores = len(os.sched_getaffinity(0))
    lx, ly, lz = cells
    # colour 0 = link-cell offset (0,0,0), basis 0: cells (4a, 4b, 4c)
    sites = [(((4 * c) * ly + 4 * b) * lx + 4 * a) * 2 for c in range(lz // 4)
             for b in range(ly // 4) for a in range(lx // 4)]
    oracle.trial(cells, model, occ, w.temperatures[0], w.seed, 0, 0, sites[0])  # warm tables
    done = 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        while time.perf_counter() - t0 < seconds and done < len(sites):
            batch = sites[done:done + 8 * cores]
            list(ex.map(lambda s: oracle.trial(cells, model, occ, w.temperatures[0], w.seed, 0, 0, s),
                        batch))
            done += len(batch)
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "attempts/s", "cores": cores, "kind": "oracle",
            "sample": f"first {done} trials of colour 0, sweep 0 of the {workload} lattice "
                      f"({w.cells[0][0]}^3 cells), FP64 energies before and after each swap"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)
    r = run_gpu(args.workload, args.precision, args.steps, args.warmup)
    w = r["w"]
    value = r["attempts"] / (r["ms"] / 1e3)
    peak, bound = PEAK[args.precision]
    avg_launch_s = (r["ms"] / 1e3) / r["launches"]
    achieved = r["flop"] / r["launches"] / avg_launch_s
    out = {
        "metric": "MC swap attempts/s",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: BCC {w.cells[0][0]}^3 cells, {sum(w.sites)} sites, "
                               f"{w.n_species} species, {w.n_in}->{w.hidden}->{w.hidden}->1 SiLU MLP, "
                               f"T={w.temperatures[0]} K",
                   "precision": args.precision, "sites": sum(w.sites)},
        "roofline": {"bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "kernel": "sweep colour kernel", "avg_launch_us": avg_launch_s * 1e6},
        "accept_ratio": r["accepts"] / max(1, r["diff"]),
        "diff_species_fraction": r["diff"] / r["attempts"],
        "fp64_recheck_fraction": r["rechecks"] / max(1, r["diff"]),
        "e_running_minus_scratch": r["e_running"] - r["e_scratch"],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
