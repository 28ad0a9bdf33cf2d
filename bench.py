"""Throughput of the swap-MC hot path: MC swap attempts per second on one MI355X.

One step = one sweep (every site attempts one nearest-neighbour swap; Sec. V-A of the
paper): all colours (mini-steps) of trial proposal, gather, features, MLP energies, dE
reduction, Metropolis decision with FP64 re-decision near the threshold, and apply.

Workload: BCC 256^3 cells (33,554,432 sites), 5 species equiatomic, 108-input one-hot MLP
108 -> 128 -> 128 -> 1 (SiLU), T = 600 K, synthetic seeded inputs (one GPU's share of the
paper's 1.009e9-atom strong-scaling system; trained weights are not available).

The headline `value` is the split-BF16 energy path (the low-precision path whose dE error
stays below 1e-4 eV); FP32, plain BF16 and FP8 are measured in the same run and reported
under "precisions" with their attempts/s, ratio to FP32, roofline fraction and error.

Prints one JSON line.  --gpus N > 1 exits: this build measures one GPU.
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

# Algorithmic work of one local energy (dense 108 -> 128 -> 128 -> 1 MLP, Eqs. (4)-(6)).
FLOP_PER_EVAL = 2 * (108 * 128 + 128 * 128 + 128)
OMEGA = 40  # local energies evaluated per different-species trial (affected zone, shells 1-3)
# Matrix-core work each precision executes per local energy (padding and split products).
EXEC_FLOP_PER_EVAL = {"fp32": 2 * (112 * 128 + 128 * 128), "bf16": 2 * (112 * 128 + 128 * 128),
                      "bf16x3": 2 * (2 * 112 * 128 + 3 * 128 * 128), "fp8": 2 * (128 * 128 + 128 * 128)}
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0, "fp8": 5000.0}
# split BF16: every product takes BF16 hi/lo parts of FP32 operands (three BF16 products per pair)
DTYPE = {"fp32": "f32", "bf16": "bf16", "bf16x3": "bf16x3", "fp8": "fp8-e4m3"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Sources that define the colour kernel; the committed traffic counters are used only while
# these files are byte-identical to the ones profiled.
KERNEL_SOURCES = ["sweep_mfma.hpp", "mfma_eval.hpp", "sweep_scalar.hpp", "lattice.hpp", "tables.hpp"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2604_08250_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(precision):
    """HBM bytes per colour-kernel launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, or None when the kernel sources changed since those counters were taken."""
    path = os.path.join(ROOT, "profiles", f"sweep_colour_{precision}_bcc256_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    return rec["traffic_bytes_per_launch"] if rec.get("kernel_source_sha256") == kernel_source_hash() else None


def colour0_sites(cells, n):
    """Trial sites of colour 0 (link-cell offset (0,0,0), basis 0) spread over the lattice."""
    lx, ly, lz = cells
    qx, qy, qz = lx // 4, ly // 4, lz // 4
    t = np.linspace(0, qx * qy * qz - 1, n).astype(np.int64)
    cx, cy, cz = t % qx, (t // qx) % qy, t // (qx * qy)
    return (((4 * cz) * ly + 4 * cy) * lx + 4 * cx) * 2


def measure(workload, precision, steps, warmup, err_samples):
    import torch

    import synth
    import paper_2604_08250_amd as smc

    w = synth.workload(workload)
    n_sites = sum(w.sites)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    mc = smc.SwapMC(w.cells, w.temperatures, w.occupancy(), w.params(), n_species=w.n_species,
                    feature=w.feature, hidden=w.hidden, precision=precision, seed=w.seed, stream=stream)
    log(f"{precision}: context ready in {time.perf_counter() - t0:.1f} s")
    if warmup:
        mc.sweep(warmup)
    torch.cuda.synchronize()
    mc.counters(reset=True)
    # ---- timed region: `steps` sweeps, inputs resident in HBM
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        mc.sweep(1)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    cnt = mc.counters(reset=True)
    attempts, diff, accepts, rechecks = (int(cnt[i].sum()) for i in range(4))
    assert attempts == n_sites * steps, (attempts, n_sites, steps)
    log(f"{precision}: {steps} sweeps in {ms:.1f} ms -> {attempts / ms * 1e3:.3e} attempts/s")
    # ---- per-kernel timing of the dominant kernel (HIP events around each launch)
    prof_sweeps = 2
    mc.profile(True)
    mc.sweep(prof_sweeps)
    colour_ms, recheck_ms, launches = mc.kernel_times()
    mc.profile(False)
    pcnt = mc.counters(reset=True)
    p_diff = int(pcnt[1].sum())
    flop = p_diff * OMEGA * FLOP_PER_EVAL
    exec_flop = p_diff * OMEGA * EXEC_FLOP_PER_EVAL[precision]
    avg_launch_s = colour_ms / 1e3 / launches
    # ---- dE error against the FP64 evaluator on trials of the next sweep's first colour
    sites = colour0_sites(w.cells[0], err_samples)
    _, dE64 = mc.delta_e64(sites)
    tr = mc.sweep(1, stats=True, trace=True)
    fast = tr["dE_fast"].cpu().numpy()[sites]
    flags = tr["flags"].cpu().numpy()[sites]
    d = (flags & 2) == 0
    err = fast[d] - dE64[d]
    # ---- local-energy and total-energy error of the precision's evaluator (final lattice)
    e_p = mc.site_energies(precision).double()
    e_64 = mc.site_energies("fp64")
    de_site = (e_p - e_64).abs()
    es, er = mc.energy()
    out = {
        "attempts_per_s": attempts / (ms / 1e3), "ms_per_sweep": ms / steps, "sweeps": steps,
        "diff_species_fraction": diff / attempts, "accept_ratio": accepts / max(diff, 1),
        "fp64_recheck_fraction": rechecks / max(diff, 1),
        "colour_kernel_us": avg_launch_s * 1e6, "recheck_kernel_ms_per_sweep": recheck_ms / prof_sweeps,
        "colour_launches": launches, "algorithmic_tflops": flop / (colour_ms / 1e3) / 1e12,
        "executed_tflops": exec_flop / (colour_ms / 1e3) / 1e12,
        "dE_err_max_eV": float(np.abs(err).max()), "dE_err_rms_eV": float(np.sqrt(np.mean(err ** 2))),
        "dE_err_trials": int(d.sum()),
        "site_energy_err_max_eV": float(de_site.max()), "site_energy_err_rms_eV": float(de_site.pow(2).mean().sqrt()),
        "energy_per_atom_err_eV": float((e_p.sum() - e_64.sum()) / n_sites),
        "running_minus_scratch_eV": float(er.sum() - es.sum()),
    }
    mc.close()
    del mc
    torch.cuda.empty_cache()
    return w, out


def measure_batched(precision="bf16", steps=3, warmup=1):
    """The 96-replica workload: one graph-replayed launch sequence per sweep over every
    replica, with the colour-kernel variant picked by the autotuner first."""
    import torch

    import synth
    import paper_2604_08250_amd as smc

    w = synth.workload("c4")
    n_sites = sum(w.sites)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    mc = smc.SwapMC(w.cells, w.temperatures, w.occupancy(), w.params(), n_species=w.n_species,
                    feature=w.feature, hidden=w.hidden, precision=precision, seed=w.seed, stream=stream)
    log(f"c4 {precision}: context ready in {time.perf_counter() - t0:.1f} s ({n_sites} sites)")
    variant, ms_var = mc.autotune()
    log(f"c4 autotune: variant {variant}, ms per variant {np.round(ms_var, 2).tolist()}")
    if warmup:
        mc.sweep(warmup)
    mc.counters(reset=True)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        mc.sweep(1)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    cnt = mc.counters(reset=True)
    attempts = int(cnt[0].sum())
    assert attempts == n_sites * steps, (attempts, n_sites, steps)
    # per-launch time of the colour kernel (HIP events around each launch, eager sweeps)
    prof_sweeps = 2
    mc.profile(True)
    mc.sweep(prof_sweeps)
    colour_ms, recheck_ms, launches = mc.kernel_times()
    mc.profile(False)
    p_diff = int(mc.counters(reset=True)[1].sum())
    alg = p_diff * OMEGA * FLOP_PER_EVAL / (colour_ms / 1e3) / 1e12
    es, er = mc.energy()
    out = {"workload": f"{len(w.cells)} replicas, cube edges {min(c[0] for c in w.cells)}..{max(c[0] for c in w.cells)}, "
                       f"{n_sites} sites, T {min(w.temperatures):.0f}..{max(w.temperatures):.0f} K",
           "precision": precision, "attempts_per_s": attempts / (ms / 1e3), "ms_per_sweep": ms / steps, "sweeps": steps,
           "graph_replay": True, "variant": int(variant), "ms_per_variant": [float(x) for x in ms_var],
           "accept_ratio": int(cnt[2].sum()) / max(int(cnt[1].sum()), 1),
           "running_minus_scratch_eV_max": float(np.abs(er - es).max()),
           "colour_launches_per_sweep": launches // prof_sweeps, "colour_kernel_ms_per_sweep": colour_ms / prof_sweeps,
           "recheck_ms_per_sweep": recheck_ms / prof_sweeps,
           "roofline": {"bound": "mfma", "achieved": alg, "peak": PEAK_TFLOPS[precision], "unit": "TFLOP/s",
                        "frac": alg / PEAK_TFLOPS[precision], "avg_launch_us": colour_ms * 1e3 / max(launches, 1)}}
    log(f"c4: {out['attempts_per_s']:.3e} attempts/s, {out['ms_per_sweep']:.1f} ms per sweep; colour kernel "
        f"{out['colour_kernel_ms_per_sweep']:.1f} ms per sweep over {out['colour_launches_per_sweep']} launches, "
        f"{alg:.1f} TFLOP/s")
    mc.close()
    del mc
    torch.cuda.empty_cache()
    return out


def measure_double_lattice(workload, precision, steps=1, warmup=0):
    """Algorithm 1 as written (sigma0/sigma1, every site evaluated before and after each
    mini-step) on the headline workload: same trajectory as the zone strategy, more work."""
    import torch

    import synth
    import paper_2604_08250_amd as smc

    w = synth.workload(workload)
    n_sites = sum(w.sites)
    stream = torch.cuda.current_stream()
    mc = smc.SwapMC(w.cells, w.temperatures, w.occupancy(), w.params(), n_species=w.n_species,
                    feature=w.feature, hidden=w.hidden, precision=precision, seed=w.seed, stream=stream)
    mc.strategy = "double_lattice"
    if warmup:
        mc.sweep(warmup)
    mc.counters(reset=True)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        mc.sweep(1)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    cnt = mc.counters(reset=True)
    attempts, diff = int(cnt[0].sum()), int(cnt[1].sum())
    assert attempts == n_sites * steps
    colours = mc.n_colours(0)
    out = {"precision": precision, "attempts_per_s": attempts / (ms / 1e3), "ms_per_sweep": ms / steps,
           "sweeps": steps, "evaluations_per_attempt": 2.0 * colours,
           "zone_evaluations_per_attempt": 40.0 * diff / attempts}
    log(f"double lattice {precision}: {out['attempts_per_s']:.3e} attempts/s, {out['ms_per_sweep']:.0f} ms per sweep")
    mc.close()
    del mc
    torch.cuda.empty_cache()
    return out


def measure_qsro(workload, steps=2, warmup=1):
    """The qSRO model (Eq. 2) on the headline lattice in FP32 with the FP64 re-decision band:
    the tiled colour kernel (each trial's region staged in LDS) evaluating neighbour counts and
    a quadratic per zone site, one site per lane, no matrix products."""
    import torch

    import synth
    import paper_2604_08250_amd as smc

    w = synth.workload(workload)
    n_sites = sum(w.sites)
    stream = torch.cuda.current_stream()
    mc = smc.SwapMC(w.cells, w.temperatures, w.occupancy(), synth.qsro_params(w.n_species), n_species=w.n_species,
                    feature=2, hidden=0, precision="fp32", seed=w.seed, stream=stream)
    if warmup:
        mc.sweep(warmup)
    mc.counters(reset=True)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        mc.sweep(1)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    cnt = mc.counters(reset=True)
    attempts = int(cnt[0].sum())
    assert attempts == n_sites * steps
    es, er = mc.energy()
    out = {"model": "qSRO (Eq. 2), shells 1-3", "precision": "fp32", "attempts_per_s": attempts / (ms / 1e3),
           "ms_per_sweep": ms / steps, "sweeps": steps,
           "accept_ratio": int(cnt[2].sum()) / max(int(cnt[1].sum()), 1),
           "running_minus_scratch_eV": float(er.sum() - es.sum())}
    log(f"qSRO fp32: {out['attempts_per_s']:.3e} attempts/s, {out['ms_per_sweep']:.1f} ms per sweep")
    mc.close()
    del mc
    torch.cuda.empty_cache()
    return out


# FCC MLPNet (Eqs. (4)-(6), 76 -> 96 -> 96 -> 96 -> 1): algorithmic work of one local energy,
# the matrix-core work each precision executes (80 padded inputs, split products), zone size.
FCC_FLOP_PER_EVAL = 2 * (76 * 96 + 2 * 96 * 96 + 96)
FCC_EXEC_FLOP_PER_EVAL = {"fp32": 2 * (80 * 96 + 2 * 96 * 96), "bf16": 2 * (80 * 96 + 2 * 96 * 96),
                          "bf16x3": 2 * (2 * 80 * 96 + 3 * 2 * 96 * 96),
                          "fp8": 2 * (128 * 96 + 2 * 128 * 96)}  # K padded to 64-wide steps
FCC_OMEGA = 28


def measure_fcc(precisions=("bf16x3", "fp32", "bf16", "fp8"), steps=2, warmup=1):
    """The paper's physical system: FCC 200^3 cells (32,000,000 sites), five species in the
    Fe29Co29Ni28Al7Ti7 proportions, the MLPNet shape (96-wide ReLU, random weights), T = 1000 K.
    Timed graph sweeps, then one profiled sweep for the zone-row kernel's average launch."""
    import torch

    import synth
    import paper_2604_08250_amd as smc

    w = synth.workload("fcc")
    n_sites = sum(w.sites)
    occ0 = w.occupancy()
    params = w.params()
    stream = torch.cuda.current_stream()
    out = {"workload": f"FCC {w.cells[0][0]}^3 cells ({n_sites} sites), Fe29Co29Ni28Al7Ti7 proportions, "
                       f"MLPNet 76-96-96-96-1 ReLU, T = {w.temperatures[0]:g} K", "precisions": {}}
    for prec in precisions:
        mc = smc.SwapMC(w.cells, w.temperatures, occ0, params, n_species=w.n_species,
                        feature=smc.SMC_FEAT_MLPNET_S12, hidden=w.hidden, precision=prec, seed=w.seed,
                        stream=stream, lattice="fcc")
        if warmup:
            mc.sweep(warmup)
        mc.counters(reset=True)
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(steps):
            mc.sweep(1)
        end.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        cnt = mc.counters(reset=True)
        attempts, diff = int(cnt[0].sum()), int(cnt[1].sum())
        assert attempts == n_sites * steps
        mc.profile(True)
        mc.sweep(1)
        rows_ms, recheck_ms, launches = mc.kernel_times()
        mc.profile(False)
        cnt1 = mc.counters(reset=True)
        rows = int(cnt1[1].sum()) * FCC_OMEGA
        # dE error against the FP64 evaluator on trials of the next sweep's first colour
        L = w.cells[0][0]
        rng = np.random.default_rng(2)
        g = rng.choice((L // 4) ** 3, size=2048, replace=False)
        gx, gy, gz = 4 * (g % (L // 4)), 4 * ((g // (L // 4)) % (L // 4)), 4 * (g // (L // 4) ** 2)
        sites = ((gz * L + gy) * L + gx) * 4  # basis 0 at link-cell offset (0,0,0): colour 0
        _, dE64 = mc.delta_e64(sites)
        tr = mc.sweep(1, stats=True, trace=True)
        fast = tr["dE_fast"].cpu().numpy()[sites]
        dsel = (tr["flags"].cpu().numpy()[sites] & 2) == 0
        err = fast[dsel] - dE64[dsel]
        mc.counters(reset=True)
        alg = rows * FCC_FLOP_PER_EVAL / (rows_ms / 1e3) / 1e12
        exe = rows * FCC_EXEC_FLOP_PER_EVAL[prec] / (rows_ms / 1e3) / 1e12
        es, er = mc.energy()
        r = {"attempts_per_s": attempts / (ms / 1e3), "ms_per_sweep": ms / steps, "sweeps": steps,
             "accept_ratio": int(cnt[2].sum()) / max(diff, 1), "recheck_frac": int(cnt[3].sum()) / max(diff, 1),
             "rows_kernel": f"fcc::k_rows_net<{prec}>", "rows_kernel_avg_us": rows_ms * 1e3 / max(launches, 1),
             "rows_kernel_share": rows_ms / max(rows_ms + recheck_ms, 1e-9),
             "rows_per_launch": rows / max(launches, 1), "algorithmic_tflops": alg, "executed_tflops": exe,
             "peak_tflops": PEAK_TFLOPS[prec], "roofline_frac": alg / PEAK_TFLOPS[prec],
             "executed_frac": exe / PEAK_TFLOPS[prec], "running_minus_scratch_eV": float(er.sum() - es.sum()),
             "dE_err_max_eV": float(np.abs(err).max()), "dE_err_rms_eV": float(np.sqrt(np.mean(err ** 2))),
             "dE_err_trials": int(dsel.sum())}
        out["precisions"][prec] = r
        log(f"FCC MLPNet {prec}: {r['attempts_per_s']:.3e} attempts/s, {r['ms_per_sweep']:.1f} ms per sweep, "
            f"rows kernel {r['rows_kernel_avg_us']:.1f} us, {alg:.1f} TFLOP/s")
        mc.close()
        del mc
        torch.cuda.empty_cache()
    fp32 = out["precisions"].get("fp32", {}).get("attempts_per_s")
    if fp32:
        for r in out["precisions"].values():
            r["speedup_vs_fp32"] = r["attempts_per_s"] / fp32
    # the qSRO model (Eq. 2) over FCC shells 1-3 on the same lattice, FP32 per-lane rows
    mc = smc.SwapMC(w.cells, w.temperatures, occ0, synth.qsro_params(w.n_species), n_species=w.n_species,
                    feature=smc.SMC_FEAT_QSRO_S123, hidden=0, precision="fp32", seed=w.seed, stream=stream,
                    lattice="fcc")
    if warmup:
        mc.sweep(warmup)
    mc.counters(reset=True)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        mc.sweep(1)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    cnt = mc.counters(reset=True)
    assert int(cnt[0].sum()) == n_sites * steps
    out["qsro_fp32"] = {"attempts_per_s": n_sites * steps / (ms / 1e3), "ms_per_sweep": ms / steps,
                        "accept_ratio": int(cnt[2].sum()) / max(int(cnt[1].sum()), 1),
                        "paper_context_attempts_per_s": {"smc_x_a100": 2.39e7, "smc_x_h100": 3.71e7,
                                                         "smc_ai_a100": 1.11e7, "smc_ai_h100": 1.87e7}}
    log(f"FCC qSRO fp32: {out['qsro_fp32']['attempts_per_s']:.3e} attempts/s, {ms / steps:.1f} ms per sweep")
    mc.close()
    del mc
    torch.cuda.empty_cache()
    # the paper's single-GPU MLPNet throughputs (its Table II, FP16 tensor cores, trained MLPNet
    # on its own FCC system): context from other hardware, not a like-for-like target -- its
    # network and zone execute about 6.8e6 flop per attempt against ~1.1e6 here
    out["paper_context_attempts_per_s"] = {"smc_x_a100": 1.59e7, "smc_x_h100": 2.47e7,
                                           "smc_ai_a100": 5.35e6, "smc_ai_h100": 7.54e6}
    return out


# Algorithmic work of one fit row: forward (Eqs. (4)-(6)) plus the backward products
# dL/dh1 = W1^T dL/dz2 (2*128*128), dW1 (2*128*128), dW0 over the 108 one-hot inputs (2*128*108)
# and the bias/output terms.
FIT_BURN_IN = 200  # sweeps of each snapshot chain before its snapshot is taken
FIT_FLOP_PER_ROW = FLOP_PER_EVAL + 2 * 128 * 128 + 2 * 128 * 128 + 2 * 128 * 108 + 4 * 128


def measure_fit(steps=5, warmup=1):
    """Fit workload: 1,024 snapshots of 16^3 cells (8.4 M rows) per step, labels from the CE
    reference Hamiltonian (computed on the GPU), BF16 forward and backward, Adam on FP32
    masters; one step = smc_fit_step (forward, loss, backward, Adam)."""
    import torch

    import synth
    import paper_2604_08250_amd as smc
    from paper_2604_08250_amd.fit import Fitter, ce_energy, sample_snapshots
    from paper_2604_08250_amd._lib import smc_energy_bwd, smc_energy_fwd

    w = synth.workload("c5")
    L, B = w.cells[0][0], w.extra["batch"]
    params0 = w.params()
    mc = smc.SwapMC([(4, 4, 4)], [1000.0], synth.random_occupancy(4, 4), params0, n_species=4,
                    feature=w.feature, hidden=w.hidden, precision="bf16", seed=0)
    # the batch: 1,024 swap-MC chains on the CE pair part from random placements, one per
    # temperature drawn uniformly in [300, 3000] K, after 200 burn-in sweeps
    ce = synth.ce_params()
    start = synth.snapshots(B, L)
    t0 = time.perf_counter()
    snaps = sample_snapshots(start, L, synth.snapshot_temperatures(B), ce["pair"], burn_in=FIT_BURN_IN, seed=0)
    torch.cuda.synchronize()
    sample_s = time.perf_counter() - t0
    labels = ce_energy(mc, ce, snaps, L)
    labels0 = ce_energy(mc, ce, torch.from_numpy(start).cuda(), L)
    log(f"c5 snapshots: {B} chains x {FIT_BURN_IN} sweeps in {sample_s:.1f} s; CE energy per atom "
        f"{float(labels0.mean()) / (2 * L ** 3):.5f} (random placements) -> {float(labels.mean()) / (2 * L ** 3):.5f} eV")
    params = torch.from_numpy(params0).cuda()
    fit = Fitter(mc, params, lr=1e-3)
    loss0 = fit.step(snaps, labels, L)
    for _ in range(max(0, warmup - 1)):
        fit.step(snaps, labels, L, want_loss=False)
    stream = torch.cuda.current_stream()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        fit.step(snaps, labels, L, want_loss=False)
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    loss1 = fit.step(snaps, labels, L)
    rows = B * 2 * L ** 3
    # forward and backward timed on their own (same inputs)
    S = torch.empty(B, dtype=torch.float64, device="cuda")
    gE = torch.full((B,), 1.0 / B, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(params)
    t = {}
    for name in ("fwd", "bwd"):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(3):
            if name == "fwd":
                smc_energy_fwd(mc.ctx, snaps.data_ptr(), B, L, params.data_ptr(), S.data_ptr())
            else:
                smc_energy_bwd(mc.ctx, snaps.data_ptr(), B, L, params.data_ptr(), gE.data_ptr(), grad.data_ptr())
        b.record(stream)
        torch.cuda.synchronize()
        t[name] = a.elapsed_time(b) / 3
    out = {"workload": f"{B} snapshots of BCC {L}^3 cells ({rows} rows), CE labels, BF16 fwd/bwd, Adam",
           "rows_per_s": rows * steps / (ms / 1e3), "ms_per_step": ms / steps, "steps": steps,
           "fwd_ms": t["fwd"], "bwd_ms": t["bwd"],
           "algorithmic_tflops": rows * FIT_FLOP_PER_ROW / (ms / steps / 1e3) / 1e12,
           "loss_first": loss0, "loss_after": loss1,
           "snapshots": f"{B} swap-MC chains on the CE pair part (qSRO blob), T ~ U[300, 3000] K, "
                        f"{FIT_BURN_IN} sweeps from random placements",
           "snapshot_sampling_s": sample_s,
           "ce_energy_per_atom_eV": {"random_placements": float(labels0.mean()) / (2 * L ** 3),
                                     "sampled": float(labels.mean()) / (2 * L ** 3)}}
    out["roofline_frac"] = out["algorithmic_tflops"] / PEAK_TFLOPS["bf16"]
    log(f"c5 fit: {out['ms_per_step']:.2f} ms per step (fwd {t['fwd']:.2f} ms, bwd {t['bwd']:.2f} ms), "
        f"loss {loss0:.3e} -> {loss1:.3e}")
    mc.close()
    del mc
    torch.cuda.empty_cache()
    return out


def _blocking(x, nblocks=10):
    """Mean and standard error of a correlated series from the spread of nblocks block means."""
    x = np.asarray(x, dtype=np.float64)
    b = x[: len(x) // nblocks * nblocks].reshape(nblocks, -1, *x.shape[1:]).mean(axis=1)
    return x.mean(axis=0), b.std(axis=0, ddof=1) / np.sqrt(nblocks)


def measure_observables(precisions=("fp64", "fp32", "bf16x3", "bf16", "fp8"), sweeps=160, burn=60, every=2):
    """Observable error of each precision against the FP64 mode on the 64^3 lattice (T = 800 K):
    the same start and Philox stream, `sweeps` sweeps, and after `burn` sweeps a sample every
    `every` sweeps of E per atom (FP64 from scratch) and the Warren-Cowley alpha of shells 1 and
    2 (the lattice average of the pair fractions of Eq. (3)); means with blocking errors.  FP32
    and split BF16 decide every trial as FP64 does (re-decision inside the guard band), so their
    chains are the FP64 chain itself; BF16 and FP8 are separate chains compared statistically."""
    import torch

    import synth
    import paper_2604_08250_amd as smc

    w = synth.workload("c2")
    occ0, params = w.occupancy(), w.params()
    n_sites = sum(w.sites)
    res, final = {}, {}
    for p in precisions:
        t0 = time.perf_counter()
        mc = smc.SwapMC(w.cells, w.temperatures, occ0, params, n_species=w.n_species, feature=w.feature,
                        hidden=w.hidden, precision=p, seed=w.seed)
        E, a1, a2 = [], [], []
        for s in range(sweeps // every):
            mc.sweep(every)
            if (s + 1) * every > burn:
                es, _ = mc.energy()
                E.append(es[0] / n_sites)
                al = mc.warren_cowley()
                a1.append(al[0])
                a2.append(al[1])
        cnt = mc.counters()
        es, er = mc.energy()
        final[p] = mc.occ.cpu().numpy()
        mE, eE = _blocking(E)
        m1, e1 = _blocking(a1)
        m2, e2 = _blocking(a2)
        res[p] = {"E_per_atom_eV": float(mE), "E_per_atom_err_eV": float(eE),
                  "alpha1": np.round(m1, 5).tolist(), "alpha1_err": np.round(e1, 5).tolist(),
                  "alpha2": np.round(m2, 5).tolist(), "alpha2_err": np.round(e2, 5).tolist(),
                  "accept_ratio": int(cnt[2].sum()) / max(int(cnt[1].sum()), 1),
                  "fp64_redecided_fraction": int(cnt[3].sum()) / max(int(cnt[1].sum()), 1),
                  "running_minus_scratch_eV": float(er[0] - es[0]), "seconds": time.perf_counter() - t0}
        mc.close()
        del mc
        torch.cuda.empty_cache()
        log(f"observables {p}: E/atom {mE:.6f} +- {eE:.6f} eV, {res[p]['seconds']:.1f} s")
    ref = res["fp64"]
    for p, r in res.items():
        if p == "fp64":
            continue
        r["chain_equals_fp64"] = bool(np.array_equal(final[p], final["fp64"]))
        r["dE_per_atom_eV"] = r["E_per_atom_eV"] - ref["E_per_atom_eV"]
        r["dE_per_atom_err_eV"] = float(np.hypot(r["E_per_atom_err_eV"], ref["E_per_atom_err_eV"]))
        for k in ("alpha1", "alpha2"):
            d = np.abs(np.asarray(r[k]) - np.asarray(ref[k]))
            e = np.hypot(np.asarray(r[k + "_err"]), np.asarray(ref[k + "_err"]))
            r[f"max_abs_d{k}"] = float(d.max())
            r[f"max_abs_d{k}_over_err"] = float((d / np.maximum(e, 1e-12)).max())
    return {"workload": f"BCC {w.cells[0][0]}^3 cells ({n_sites} sites), {w.n_species} species, "
                        f"T = {w.temperatures[0]:g} K, {sweeps} sweeps, samples every {every} after {burn}",
            "precisions": res}


def cpu_baseline(workload, seconds=12.0, cores=None):
    """The FP64 oracle, unchanged, on a bounded sample: the first trials of colour 0 of
    sweep 0 of the same workload, run on all host cores through a thread pool."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    import synth

    w = synth.workload(workload)
    cells = w.cells[0]
    occ = w.occupancy()
    model = oracle.MLP(w.feature, w.hidden, w.params())
    cores = cores or len(os.sched_getaffinity(0))
    lx, ly, lz = cells
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
            "sample": f"first {done} trials of colour 0 of sweep 0 of the {cells[0]}^3-cell lattice "
                      f"(FP64 energies of the 40-site zone before and after each swap)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--precision", default="bf16x3")
    ap.add_argument("--others", default="fp32,bf16,fp8")
    ap.add_argument("--other-steps", type=int, default=3)
    ap.add_argument("--err-samples", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the 96-replica measurement")
    ap.add_argument("--no-fit", action="store_true", help="skip the fit-step measurement")
    ap.add_argument("--no-double-lattice", action="store_true", help="skip the double-lattice measurement")
    ap.add_argument("--no-qsro", action="store_true", help="skip the qSRO-model measurement")
    ap.add_argument("--no-fcc", action="store_true", help="skip the FCC MLPNet measurement")
    ap.add_argument("--no-observables", action="store_true", help="skip the per-precision observable chains")
    ap.add_argument("--only", choices=["batched", "fit", "qsro", "fcc", "observables"], default=None,
                    help="run only this measurement and print its object (for profiling)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run 4 plain device copies of this many GiB (scale for the HBM byte counters)")
    ap.add_argument("--print-kernel-hash", action="store_true",
                    help="print the hash of the colour-kernel sources (recorded with traffic counters)")
    args = ap.parse_args()
    if args.print_kernel_hash:
        print(kernel_source_hash())
        return
    if args.copy_calibration > 0:
        import torch
        n = int(args.copy_calibration * 2**30) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each": n * 4, "copies": 4}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not part of this build.", file=sys.stderr)
        sys.exit(2)
    if args.only:
        if args.only == "batched":
            res = measure_batched(steps=args.steps, warmup=args.warmup)
        elif args.only == "fit":
            res = measure_fit(steps=args.steps, warmup=args.warmup)
        elif args.only == "observables":
            res = measure_observables()
        elif args.only == "fcc":
            res = measure_fcc(tuple(x for x in args.precision.split(",") if x), steps=args.steps,
                              warmup=args.warmup)
        else:
            res = measure_qsro(args.workload, steps=args.steps, warmup=args.warmup)
        print(json.dumps({args.only: res}), flush=True)
        return
    w, head = measure(args.workload, args.precision, args.steps, args.warmup, args.err_samples)
    precs = {args.precision: head}
    for p in [x for x in args.others.split(",") if x and x != args.precision]:
        precs[p] = measure(args.workload, p, args.other_steps, 1, args.err_samples)[1]
    fp32 = precs.get("fp32", {}).get("attempts_per_s")
    for p, r in precs.items():
        r["peak_tflops"] = PEAK_TFLOPS[p]
        r["roofline_frac"] = r["algorithmic_tflops"] / PEAK_TFLOPS[p]
        r["executed_frac"] = r["executed_tflops"] / PEAK_TFLOPS[p]
        if fp32:
            r["speedup_vs_fp32"] = r["attempts_per_s"] / fp32
        r["dE_err_below_1e-4_eV"] = r["dE_err_max_eV"] < 1e-4
    value = head["attempts_per_s"]
    out = {
        "metric": "MC swap attempts/s",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_sweep"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": f"BCC {w.cells[0][0]}^3 cells ({sum(w.sites)} sites), {w.n_species} species "
                               f"equiatomic, one-hot {w.n_in}-{w.hidden}-{w.hidden}-1 SiLU MLP, "
                               f"T = {w.temperatures[0]:g} K, {args.precision} energy path",
                   "precision": args.precision, "sites": sum(w.sites)},
        "roofline": {"bound": "mfma", "achieved": head["algorithmic_tflops"], "peak": PEAK_TFLOPS[args.precision],
                     "unit": "TFLOP/s", "frac": head["roofline_frac"],
                     "traffic": measured_traffic(args.precision) if args.workload == "c3" else None,
                     "kernel": f"k_sweep_colour_mfma<{args.precision}>",
                     "avg_launch_us": head["colour_kernel_us"], "executed_frac": head["executed_frac"]},
        "precisions": precs,
    }
    if not args.no_double_lattice:
        dl = measure_double_lattice(args.workload, args.precision)
        dl["zone_over_double_lattice"] = head["attempts_per_s"] / dl["attempts_per_s"]
        out["double_lattice"] = dl
    if not args.no_qsro:
        out["qsro"] = measure_qsro(args.workload)
    if not args.no_fcc:
        out["fcc"] = measure_fcc()
    if not args.no_batched:
        out["batched"] = measure_batched()
    if not args.no_fit:
        out["fit"] = measure_fit()
    if not args.no_observables:
        out["observables"] = measure_observables()
    # context, not a target: the paper's record run (Table I; Sec. V-B), 4e12 atoms of its FCC
    # alloy with the qSRO model on 2,048 Ascend 910 NPUs (4,096 dies)
    out["paper_context"] = {"record_run_attempts_per_s": 3.77e10, "record_run_atoms": 4.0e12,
                            "record_run_devices": "2,048 Ascend 910 NPUs (4,096 dies)",
                            "record_run_per_die_attempts_per_s": 3.77e10 / 4096, "record_run_model": "qSRO, FCC"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.cpu_seconds)
        one = cpu_baseline(args.workload, args.cpu_seconds / 2, cores=1)
        out["cpu_baseline"]["one_core"] = {"value": one["value"], "unit": one["unit"], "sample": one["sample"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
