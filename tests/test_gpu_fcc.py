"""The FCC path (MLPNet of Eqs. (4)-(6) on the matrix cores, qSRO per lane) against the FCC
oracle, through the C ABI.

Bar: FP64 local energies within 1e-12 relative of the oracle; FP32 and split BF16 within
1e-5 / 2e-4 eV of it; BF16 within 1e-4 eV of a CPU emulation of its quantisation points.
Sweeps: decisions equal to the oracle's except within 1e-9 eV of the threshold, FP32 |dE|
error below 1e-5 eV, FP64 re-decided dE within 1e-9 eV; FP64 mode equal trial for trial;
graph replays equal per-launch sweeps bit for bit; running totals equal from-scratch totals
and the oracle's."""
import numpy as np
import pytest

import synth
from emulate import mlpnet_emulate
from gpu_common import DECISION_BAND_EV, need_gpu, trace_to_numpy
from oracle import fcc

pytestmark = pytest.mark.gpu

H = 96


def _banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _make(cells_list, temps, model="mlpnet", precision="fp32", n_species=5, seed=7, comp=synth.HEA_COMPOSITION,
          params=None, guard_eV=-1.0):
    import paper_2604_08250_amd as smc
    occ = np.concatenate([synth.random_occupancy(c, n_species, comp, seed=30 + r, basis=4)
                          for r, c in enumerate(cells_list)])
    if model == "mlpnet":
        p = synth.mlpnet_params(H) if params is None else params
        feat, hid, om = smc.SMC_FEAT_MLPNET_S12, H, fcc.MLPNet(H, p)
    else:
        p = synth.qsro_params(n_species=n_species) if params is None else params
        feat, hid, om = smc.SMC_FEAT_QSRO_S123, 0, fcc.QSRO(p)
    mc = smc.SwapMC(cells_list, temps, occ, p, n_species=n_species, feature=feat, hidden=hid, precision=precision,
                    seed=seed, lattice="fcc", guard_eV=guard_eV)
    return mc, om, occ


def _slices(cells_list):
    out, s0 = [], 0
    for c in cells_list:
        n = 4 * int(np.prod(c))
        out.append(slice(s0, s0 + n))
        s0 += n
    return out


def _cache_offset(mc):
    """Per replica sum over sites of (cache - FP64 local energy): the sweep precision's error."""
    ec = mc.ecache.cpu().numpy().astype(np.float64)
    e64 = mc.site_energies("fp64").cpu().numpy()
    return np.array([float((ec[s] - e64[s]).sum()) for s in _slices([tuple(c) for c in mc.cells])])


def _check_running_total(mc, d0, accepts, rechecks, per_recheck):
    """The running total adds each accepted trial's deciding dE while the cache takes the sweep
    precision's zone energies, so running - FP64 total = (cache offset now - at the start)
    + FP32 rounding of the zone sums + (FP64 - fast dE) of the re-decided accepted trials.
    Both remainders are sums of terms of random sign: the bound takes each term at its largest
    size (1e-6 eV for a 28-term FP32 sum, the precision's largest dE error for a re-decision)
    times the square root of the number of terms."""
    es, er = mc.energy()
    d1 = _cache_offset(mc)
    for r in range(len(es)):
        tol = 1e-6 * float(accepts[r]) ** 0.5 + per_recheck * float(rechecks[r]) ** 0.5 + 1e-9
        assert abs((er[r] - es[r]) - (d1[r] - d0[r])) < tol, (r, er[r] - es[r], d1[r] - d0[r], tol)


def _compare_sweep(cells, model, occ_or, T, seed, replica, sweep, tr, gpu_occ, de_tol):
    """One oracle sweep against the GPU's.  A decision that differs is tolerated only within
    DECISION_BAND_EV of the threshold; the oracle sweep is then run again from the same start
    with the GPU's decision imposed on exactly those trials, and the lattice and every other
    decision must agree.  Returns (oracle stats of the final run, tolerated disagreements)."""
    start = occ_or.copy()
    flags = tr["flags"]
    same = (flags & 2).astype(bool)
    acc_gpu = (flags & 1).astype(bool)
    force = np.full(occ_or.size, -1, dtype=np.int8)
    tolerated = 0
    for _ in range(64):
        occ_or[:] = start
        st, ref = fcc.sweep(cells, model, occ_or, T, seed, replica, sweep, trace=True, nthreads=8,
                            force=force if tolerated else None)
        assert np.array_equal(same, ref["same"].astype(bool))
        diff = np.nonzero(acc_gpu != ref["accept"].astype(bool))[0]
        if diff.size == 0:
            break
        for s in diff:
            gap = abs(ref["dE"][s] - ref["theta"][s])
            assert force[s] < 0 and gap < DECISION_BAND_EV, (sweep, s, ref["dE"][s], ref["theta"][s], tr["dE"][s])
            force[s] = 1 if acc_gpu[s] else 0
            tolerated += 1
    else:
        raise AssertionError("forced re-runs of the oracle sweep did not converge")
    assert np.array_equal(gpu_occ, occ_or), f"occupancy differs after sweep {sweep}"
    d = ~ref["same"].astype(bool)
    if de_tol is not None:
        err = np.abs(tr["dE_fast"][d] - ref["dE"][d])
        assert err.max(initial=0.0) < de_tol, err.max()
    fp64 = d & ((flags & 4) != 0)
    if fp64.any():
        assert np.abs(tr["dE"][fp64] - ref["dE"][fp64]).max() < 1e-9
    return st, tolerated


@pytest.mark.parametrize("prec,tol", [("fp64", None), ("fp32", 1e-5), ("bf16x3", 2e-4), ("bf16", None),
                                      ("fp8", None)])
def test_fcc_site_energies(prec, tol):
    need_gpu()
    _banner(f"fcc site energies {prec}")
    cells = (5, 6, 9)
    mc, model, occ = _make([cells], [1000.0])
    e = mc.site_energies(prec).cpu().numpy().astype(np.float64)
    want = fcc.all_site_energies(cells, model, occ)
    if prec == "fp64":
        np.testing.assert_allclose(e, want, rtol=1e-12, atol=1e-12)
    elif prec == "bf16":
        X = np.stack([fcc.features(cells, occ, j) for j in range(occ.size)])
        emu = mlpnet_emulate(synth.mlpnet_params(H), X, "bf16")
        # a BF16 activation can round the other way when FP32 sums differ in the last bit
        assert np.linalg.norm(e - emu) / np.linalg.norm(emu) < 1e-4
        assert np.abs(e - emu).max() < 1e-2
        assert np.abs(e - want).max() < 0.05
    elif prec == "fp8":
        X = np.stack([fcc.features(cells, occ, j) for j in range(occ.size)])
        emu = mlpnet_emulate(synth.mlpnet_params(H), X, "fp8")
        d_emu, d_emu64 = np.abs(e - emu), np.abs(emu - want)
        _banner(f"fcc fp8: |gpu-emu| rms {np.sqrt((d_emu ** 2).mean()):.3e}, |emu-fp64| rms "
                f"{np.sqrt((d_emu64 ** 2).mean()):.3e}, |gpu-fp64| max {np.abs(e - want).max():.3e}")
        # an E4M3 activation can round the other way when FP32 sums differ in the last bit: the
        # disagreement must stay far below the precision's own error
        assert np.sqrt((d_emu ** 2).mean()) < 0.1 * np.sqrt((d_emu64 ** 2).mean())
        assert np.median(d_emu) < 0.05 * np.median(d_emu64) + 1e-6
    else:
        assert np.abs(e - want).max() < tol
        X = np.stack([fcc.features(cells, occ, j) for j in range(0, occ.size, 7)])
        emu = mlpnet_emulate(synth.mlpnet_params(H), X, prec)
        assert np.abs(e[::7] - emu).max() < 2e-5
    mc.close()


@pytest.mark.parametrize("prec,de_tol", [("fp32", 1e-5), ("bf16x3", 2.5e-5), ("fp64", None)])
def test_fcc_mlpnet_sweeps_match_oracle(prec, de_tol):
    # de_tol: the dE error of the sweep precision stays below a quarter of its default guard
    """Two replicas (one with ragged link cells), four sweeps each."""
    need_gpu()
    cells_list = [(8, 8, 8), (5, 6, 9)]
    temps = [900.0, 2000.0]
    mc, model, occ = _make(cells_list, temps, precision=prec)
    _banner(f"fcc mlpnet sweeps {prec}")
    sl = _slices(cells_list)
    ors = [occ[s].copy() for s in sl]
    d0 = _cache_offset(mc)
    tot_attempts = 0
    for t in range(4):
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        now = mc.occ.cpu().numpy()
        for r, (cells, s) in enumerate(zip(cells_list, sl)):
            sub = {k: (v[s] if isinstance(v, np.ndarray) and v.size == now.size else v) for k, v in tr.items()}
            st, _ = _compare_sweep(cells, model, ors[r], temps[r], 7, r, t, sub, now[s], de_tol)
            assert int(tr["attempts"][r]) == st.attempts == now[s].size
            assert int(tr["diff_species"][r]) == st.diff_species
        tot_attempts += int(tr["attempts"].sum())
    es, er = mc.energy()
    for r, (cells, s) in enumerate(zip(cells_list, sl)):
        want = fcc.total_energy(cells, model, ors[r])
        assert es[r] == pytest.approx(want, abs=1e-8)
        if prec == "fp64":  # every decision and every dE added in FP64
            assert er[r] == pytest.approx(want, abs=1e-6)
    c = mc.counters()
    if prec != "fp64":
        _check_running_total(mc, d0, c[2], c[3], 2e-4)
    if prec == "fp64":
        c = mc.counters()
        assert np.array_equal(c[3], c[1])  # every different-species trial re-decided in FP64
    mc.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_fcc_low_precision_follows_its_own_energies(prec):
    """BF16 and FP8 decisions follow their own dE outside the guard band; the running total
    keeps the accounting identity with the cache offset."""
    need_gpu()
    _banner(f"fcc {prec} sweeps")
    cells = (8, 8, 8)
    mc, model, occ = _make([cells], [1200.0], precision=prec)
    d0 = _cache_offset(mc)
    for t in range(3):
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        flags = tr["flags"]
        d = (flags & 2) == 0
        fast = d & ((flags & 4) == 0)
        acc = (flags & 1).astype(bool)
        # theta from the oracle's proposal of each trial site
        th = np.array([fcc.propose(7, s, t, 0)[1] for s in np.nonzero(fast)[0]])
        theta = -synth_kb() * 1200.0 * np.log(th)
        assert np.array_equal(acc[fast], tr["dE"][fast] <= theta)
    es, er = mc.energy()
    assert es[0] == pytest.approx(fcc.total_energy(cells, model, mc.occ.cpu().numpy()), abs=1e-8)
    c = mc.counters()
    _check_running_total(mc, d0, c[2], c[3], {"bf16": 5e-2, "fp8": 0.5}[prec])
    mc.close()


def synth_kb():
    from oracle import KB_EV_PER_K
    return KB_EV_PER_K


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fcc_qsro_sweeps_match_oracle(prec):
    need_gpu()
    cells_list = [(6, 6, 6), (4, 5, 9)]
    temps = [700.0, 1500.0]
    mc, model, occ = _make(cells_list, temps, model="qsro", precision=prec)
    _banner(f"fcc qsro sweeps {prec}")
    sl = _slices(cells_list)
    ors = [occ[s].copy() for s in sl]
    d0 = _cache_offset(mc)
    for t in range(4):
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        now = mc.occ.cpu().numpy()
        for r, (cells, s) in enumerate(zip(cells_list, sl)):
            sub = {k: (v[s] if isinstance(v, np.ndarray) and v.size == now.size else v) for k, v in tr.items()}
            _compare_sweep(cells, model, ors[r], temps[r], 7, r, t, sub, now[s], 1e-5 if prec == "fp32" else None)
    es, er = mc.energy()
    for r, (cells, s) in enumerate(zip(cells_list, sl)):
        assert es[r] == pytest.approx(fcc.total_energy(cells, model, ors[r]), abs=1e-9)
        if prec == "fp64":
            assert er[r] == pytest.approx(es[r], abs=1e-7)
    if prec == "fp32":
        c = mc.counters()
        _check_running_total(mc, d0, c[2], c[3], 1e-5)
    mc.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16", "fp8"])
def test_fcc_graph_replays_equal_per_launch(prec):
    need_gpu()
    import torch
    _banner(f"fcc graph vs per-launch {prec}")
    a = _make([(8, 8, 8), (4, 4, 4)], [800.0, 1600.0], precision=prec)[0]
    b = _make([(8, 8, 8), (4, 4, 4)], [800.0, 1600.0], precision=prec)[0]
    a.use_graph(True)
    b.use_graph(False)
    for _ in range(3):
        a.sweep(2)
        torch.cuda.synchronize()
        b.sweep(2)
        assert np.array_equal(a.occ.cpu().numpy(), b.occ.cpu().numpy())
        assert np.array_equal(a.ecache.cpu().numpy(), b.ecache.cpu().numpy())
    assert np.array_equal(a.counters(), b.counters())
    a.close()
    b.close()


def test_fcc_warren_cowley_and_l12():
    need_gpu()
    import paper_2604_08250_amd as smc
    _banner("fcc warren-cowley")
    cells = (6, 5, 7)
    mc, model, occ = _make([cells, (4, 4, 4)], [500.0, 500.0], model="qsro")
    mc.sweep(3)
    now = mc.occ.cpu().numpy()
    for r, (c, s) in enumerate(zip([cells, (4, 4, 4)], _slices([cells, (4, 4, 4)]))):
        np.testing.assert_allclose(mc.warren_cowley(r), fcc.warren_cowley(c, now[s], 5), rtol=0, atol=1e-14)
    mc.close()
    # L1_2 A3B: alpha_1^{AB} = -1/3, alpha_2^{AB} = 1 (closed forms)
    l12 = (np.arange(4 * 64) % 4 == 0).astype(np.uint8)
    mc = smc.SwapMC([(4, 4, 4)], [500.0], l12, synth.qsro_params(2), n_species=2, feature=smc.SMC_FEAT_QSRO_S123,
                    hidden=0, lattice="fcc")
    a = mc.warren_cowley(0)
    assert a[0, 0, 1] == pytest.approx(-1 / 3) and a[1, 0, 1] == pytest.approx(1.0)
    mc.close()


def test_fcc_unsupported_configurations():
    need_gpu()
    import paper_2604_08250_amd as smc
    _banner("fcc unsupported")
    occ = synth.random_occupancy((4, 4, 4), 4, None, seed=1, basis=4)
    with pytest.raises(smc.SMCError):  # qSRO on FCC runs in FP32 or FP64
        smc.SwapMC([(4, 4, 4)], [800.0], occ, synth.qsro_params(4), n_species=4, feature=smc.SMC_FEAT_QSRO_S123,
                   hidden=0, precision="fp8", lattice="fcc")
    with pytest.raises(smc.SMCError):  # the MLPNet is 96 wide
        smc.SwapMC([(4, 4, 4)], [800.0], occ, synth.mlpnet_params(64), n_species=4, feature=smc.SMC_FEAT_MLPNET_S12,
                   hidden=64, lattice="fcc")
    with pytest.raises(smc.SMCError):  # the BCC one-hot model has no FCC form
        smc.SwapMC([(4, 4, 4)], [800.0], occ, synth.mlp_params(108, 128), n_species=4,
                   feature=smc.SMC_FEAT_ONEHOT_S123, hidden=128, lattice="fcc")
    mc = _make([(4, 4, 4)], [800.0])[0]
    with pytest.raises(smc.SMCError):
        mc.strategy = "double_lattice"
    mc.close()


def test_fcc_full_size_sampled():
    """200^3 cells (32,000,000 sites), the benchmark's workload: sampled cache entries and FP64
    local energies against the oracle one by one, then one sweep; the running total stays
    equal to the from-scratch total and every site is attempted once."""
    need_gpu()
    _banner("fcc full size 200^3 sampled")
    cells = (200, 200, 200)
    w = synth.workload("fcc")
    occ = w.occupancy()
    import paper_2604_08250_amd as smc
    p = w.params()
    model = fcc.MLPNet(H, p)
    mc = smc.SwapMC(w.cells, w.temperatures, occ, p, n_species=5, feature=smc.SMC_FEAT_MLPNET_S12, hidden=H,
                    precision="bf16x3", seed=w.seed, lattice="fcc")
    rng = np.random.default_rng(5)
    sample = rng.integers(occ.size, size=300)
    ec = mc.ecache.cpu().numpy()[sample].astype(np.float64)
    e64 = mc.site_energies("fp64").cpu().numpy()[sample]
    want = np.array([fcc.site_energy(cells, model, occ, int(j)) for j in sample])
    assert np.abs(e64 - want).max() < 1e-12 * max(1.0, np.abs(want).max())
    assert np.abs(ec - want).max() < 2e-4
    d0 = _cache_offset(mc)
    st = mc.sweep(1, stats=True)
    assert int(st["attempts"][0]) == occ.size
    _check_running_total(mc, d0, st["accepts"], st["rechecks"], 2e-4)
    now = mc.occ.cpu().numpy()
    assert np.array_equal(np.bincount(now, minlength=5), np.bincount(occ, minlength=5))
    mc.close()


@pytest.mark.parametrize("case", ["T0", "Tinf", "one_species", "binary"])
def test_fcc_degenerate_cases(case):
    """T = 0 (only dE <= 0 accepted), T = +inf (every different-species swap accepted), a lattice
    of one species (no trial is evaluated: the active list stays empty) and a binary alloy, each
    against the oracle for three sweeps."""
    need_gpu()
    import paper_2604_08250_amd as smc
    _banner(f"fcc degenerate {case}")
    cells = (4, 5, 6)
    T = {"T0": 0.0, "Tinf": float("inf")}.get(case, 900.0)
    if case == "one_species":
        occ = np.full(4 * int(np.prod(cells)), 2, dtype=np.uint8)
        S = 3
    elif case == "binary":
        occ = synth.random_occupancy(cells, 2, [0.75, 0.25], seed=12, basis=4)
        S = 2
    else:
        occ = synth.random_occupancy(cells, 5, synth.HEA_COMPOSITION, seed=13, basis=4)
        S = 5
    p = synth.mlpnet_params(H)
    model = fcc.MLPNet(H, p)
    mc = smc.SwapMC([cells], [T], occ, p, n_species=S, feature=smc.SMC_FEAT_MLPNET_S12, hidden=H, precision="fp32",
                    seed=3, lattice="fcc")
    ref = occ.copy()
    for t in range(3):
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        st, _ = _compare_sweep(cells, model, ref, T, 3, 0, t, tr, mc.occ.cpu().numpy(), 1e-5)
        assert int(tr["attempts"][0]) == occ.size
        if case == "one_species":
            assert int(tr["diff_species"][0]) == 0 and int(tr["accepts"][0]) == 0
            assert np.all(tr["flags"] == 2)
        if case == "Tinf":
            assert int(tr["accepts"][0]) == int(tr["diff_species"][0])
        if case == "T0":
            acc = (tr["flags"] & 1).astype(bool)
            assert np.all(tr["dE"][acc] <= 0.0)
    es, er = mc.energy()
    assert es[0] == pytest.approx(fcc.total_energy(cells, model, ref), abs=1e-8)
    assert np.array_equal(np.bincount(mc.occ.cpu().numpy(), minlength=S), np.bincount(occ, minlength=S))
    mc.close()


@pytest.mark.parametrize("kind", ["mlpnet", "qsro"])
def test_fcc_fp64_probe_matches_oracle(kind):
    """smc_delta_e64 on FCC: the partner of each trial site's proposal and the FP64 dE of that
    swap on the current lattice, against the oracle's proposal and dE; nothing changes."""
    need_gpu()
    _banner(f"fcc fp64 probe {kind}")
    cells = (5, 6, 9)
    mc, model, occ = _make([cells], [900.0], model=kind)
    mc.sweep(2)
    now = mc.occ.cpu().numpy().copy()
    ec = mc.ecache.cpu().numpy().copy()
    rng = np.random.default_rng(8)
    sites = rng.choice(now.size, size=200, replace=False)
    partners, d64 = mc.delta_e64(sites, sweep=5)
    for s, p, d in zip(sites, partners, d64):
        dir_, _ = fcc.propose(7, int(s), 5, 0)
        assert p == fcc.neighbor(cells, int(s), dir_)
        want = 0.0 if now[s] == now[p] else fcc.delta_e(cells, model, now, int(s), int(p))
        assert d == pytest.approx(want, abs=1e-10)
    assert np.array_equal(mc.occ.cpu().numpy(), now) and np.array_equal(mc.ecache.cpu().numpy(), ec)
    mc.close()


def test_fcc_set_params_and_resume():
    """New weights through smc_set_params (the captured sweep holds the output bias, so it must be
    rebuilt) give the oracle's energies and sweeps; a fresh context resumed at the same sweep
    index from the same lattice continues the same chain."""
    need_gpu()
    import paper_2604_08250_amd as smc
    _banner("fcc set_params and resume")
    cells = (6, 5, 4)
    a, model, occ = _make([cells], [900.0], precision="fp32")
    a.use_graph(True)
    a.sweep(2)
    p2 = synth.mlpnet_params(H, seed=21)
    a.set_params(p2)
    m2 = fcc.MLPNet(H, p2)
    now = a.occ.cpu().numpy().copy()
    np.testing.assert_allclose(a.site_energies("fp64").cpu().numpy(), fcc.all_site_energies(cells, m2, now),
                               rtol=1e-12, atol=1e-12)
    b = smc.SwapMC([cells], [900.0], now, p2, n_species=5, feature=smc.SMC_FEAT_MLPNET_S12, hidden=H,
                   precision="fp32", seed=7, lattice="fcc")
    b.sweep_index = a.sweep_index
    ref = now.copy()
    for t in range(2):
        a.sweep(1)
        tr = trace_to_numpy(b.sweep(1, stats=True, trace=True))
        _compare_sweep(cells, m2, ref, 900.0, 7, 0, 2 + t, tr, b.occ.cpu().numpy(), 1e-5)
        assert np.array_equal(a.occ.cpu().numpy(), b.occ.cpu().numpy())
    a.close()
    b.close()
