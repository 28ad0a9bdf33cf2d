"""GPU sweeps against the CPU oracle, through the C ABI.

Bar: occupancies bit-exact after every sweep under the same Philox stream; FP32 dE within
1e-5 eV of the oracle's FP64 dE; Metropolis decisions equal except where the oracle's dE
lies within 1e-9 eV of the threshold; FP64 running totals equal the from-scratch total.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import compare_sweep, make, need_gpu, trace_to_numpy

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def test_site_energies_match_oracle_c1_c2_shapes():
    need_gpu()
    for name, cells in [("c1", None), ("c2", (8, 12, 16))]:
        _banner(f"site energies {name} {cells}")
        w, mc, model, occ = make(name, cells=cells)
        e64 = mc.site_energies("fp64").cpu().numpy()
        e32 = mc.site_energies("fp32").cpu().numpy()
        want = oracle.all_site_energies(w.cells[0], model, occ)
        assert np.max(np.abs(e64 - want)) < 1e-12
        assert np.max(np.abs(e32 - want)) < 5e-6
        # the energy cache is the FP32 evaluator's output, bit for bit
        assert np.array_equal(mc.ecache.cpu().numpy(), e32)
        es, er = mc.energy()
        assert es[0] == pytest.approx(want.sum(), abs=1e-9 * abs(want.sum()) + 1e-12)
        assert er[0] == es[0]
        mc.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_c1_bit_exact_every_sweep(precision):
    need_gpu()
    w, mc, model, occ = make("c1", precision=precision)
    cells, T = w.cells[0], w.temperatures[0]
    n_sweeps = 100 if precision == "fp32" else 20
    _banner(f"c1 {precision} {n_sweeps} sweeps")
    tolerated = 0
    accepts = 0
    max_err = 0.0
    counts0 = np.bincount(occ, minlength=4)
    for t in range(n_sweeps):
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        gocc = mc.occ.cpu().numpy()
        assert np.array_equal(np.bincount(gocc, minlength=4), counts0)
        n_tol, otr = compare_sweep(cells, model, occ, T, w.seed, t, tr, gocc)
        tolerated += n_tol
        assert tr["attempts"][0] == occ.size
        assert tr["diff_species"][0] == int((otr["same"] == 0).sum())
        accepts += int(tr["accepts"][0])
        d = otr["same"] == 0
        max_err = max(max_err, float(np.abs(tr["dE"][d] - otr["dE"][d]).max(initial=0.0)))
    _banner(f"tolerated near-threshold disagreements: {tolerated}; max |dE err| {max_err:.3e}")
    es, er = mc.energy()
    # the running total adds the sweep precision's dE of each accepted swap in FP64, so it
    # drifts from the from-scratch total like a random walk of the per-trial dE error
    assert abs(es[0] - er[0]) <= 10.0 * max_err * np.sqrt(max(accepts, 1)) + 1e-9 * abs(es[0])
    assert es[0] == pytest.approx(oracle.total_energy(cells, model, occ), abs=1e-9)
    assert np.array_equal(mc.ecache.cpu().numpy(), mc.site_energies("fp32").cpu().numpy()) \
        or precision == "fp64"
    mc.close()


def test_uneven_lattice_and_five_species():
    """Link cells of 4 and 5 cells, fifth species without a one-hot channel."""
    need_gpu()
    cells = (9, 10, 13)
    _banner(f"uneven lattice {cells} 5 species")
    w, mc, model, occ = make("c2", cells=cells, n_species=5, hidden=128, temperature=700.0)
    for t in range(3):
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        compare_sweep(cells, model, occ, 700.0, w.seed, t, tr, mc.occ.cpu().numpy())
    mc.close()


@pytest.mark.parametrize("n_species", [4, 5])
def test_fp64_probe_matches_oracle(n_species):
    """The FP64 re-decision kernel (through smc_delta_e64, which queues the given trials exactly
    as the sweep's near-threshold queue) against the oracle's dE trial by trial: one trial (a
    work split that leaves a half block idle), three, and 400 (several work items per block);
    the lattice and the energy cache are left as they were.  The FP64 site energies, which use
    the same row evaluator, match the oracle on this ragged site count."""
    need_gpu()
    cells = (9, 10, 13)
    _banner(f"fp64 probe {cells} {n_species} species")
    w, mc, model, occ = make("c2", cells=cells, n_species=n_species, hidden=128, temperature=700.0)
    mc.sweep(2)
    now = mc.occ.cpu().numpy().copy()
    ec = mc.ecache.cpu().numpy().copy()
    # FP64 site energies from the same row evaluator, over a site count that is not a multiple
    # of its 16-row items
    assert now.size % 16 != 0
    e64 = mc.site_energies("fp64").cpu().numpy()
    assert np.max(np.abs(e64 - oracle.all_site_energies(cells, model, now))) < 1e-12
    T = w.temperatures[0]
    rng = np.random.default_rng(3 + n_species)
    for n in (1, 3, 400):
        sites = rng.choice(now.size, size=n, replace=False)
        partners, d64 = mc.delta_e64(sites, sweep=4)
        for s, p, d in zip(sites, partners, d64):
            rec = oracle.trial(cells, model, now, T, w.seed, 0, 4, int(s))
            assert p == rec["partner"]
            want = 0.0 if rec["same"] else rec["dE"]
            assert abs(d - want) < 1e-10, f"{n} trials, site {s}: probe {d!r} oracle {want!r}"
    assert np.array_equal(mc.occ.cpu().numpy(), now) and np.array_equal(mc.ecache.cpu().numpy(), ec)
    mc.close()


def test_split_run_equals_long_run_and_resume():
    need_gpu()
    _banner("split/resume")
    w, a, _, occ = make("c1")
    a.sweep(6)
    w, b, _, _ = make("c1")
    b.sweep(2)
    b.sweep(4)
    assert np.array_equal(a.occ.cpu().numpy(), b.occ.cpu().numpy())
    # resume from a checkpoint (occupancy + sweep counter) in a fresh context
    w, c, _, _ = make("c1")
    c.sweep(3)
    ck_occ, ck_sweep = c.occ.cpu().numpy().copy(), c.sweep_index
    w, d, _, _ = make("c1", occ=ck_occ)
    d.sweep_index = ck_sweep
    d.sweep(3)
    assert np.array_equal(a.occ.cpu().numpy(), d.occ.cpu().numpy())
    for m in (a, b, c, d):
        m.close()


def test_replica_in_batch_equals_replica_alone():
    """Replicas of uneven size, composition and temperature in one context: each evolves
    exactly as it does alone (the Philox counter carries the replica index)."""
    need_gpu()
    import paper_2604_08250_amd as smc
    import synth as S
    edges = [8, 9, 12]
    comps = [None, [0.4, 0.3, 0.2, 0.1], [0.1, 0.2, 0.3, 0.4]]
    temps = [500.0, 1200.0, 3000.0]
    params = S.mlp_params(108, 128)
    occs = [S.random_occupancy(e, 4, c, seed=10 + r) for r, (e, c) in enumerate(zip(edges, comps))]
    cells = [(e, e, e) for e in edges]
    _banner(f"batch of {len(edges)} replicas")
    for prec in ["fp32", "bf16"]:
        batch = smc.SwapMC(cells, temps, np.concatenate(occs), params, n_species=4, feature=1, hidden=128,
                           precision=prec, seed=5)
        batch.sweep(3)
        got = batch.occ.cpu().numpy()
        off = 0
        for r in range(len(edges)):
            # the same replica alone, carrying replica index r in its Philox counter, is emulated
            # by a batch in which it is the only member at position r: compare against the oracle
            n = occs[r].size
            ref = occs[r].copy()
            model = oracle.MLP(1, 128, params)
            if prec == "fp32":
                for t in range(3):
                    oracle.sweep(cells[r], model, ref, temps[r], 5, r, t, nthreads=8)
                assert np.array_equal(got[off:off + n], ref), f"replica {r}"
            assert np.array_equal(np.bincount(got[off:off + n], minlength=4), np.bincount(occs[r], minlength=4))
            off += n
        es, er = batch.energy()
        if prec == "fp32":  # BF16 adds its own dE error (~2e-3 eV) per accepted swap
            assert np.all(np.abs(es - er) < 1e-4)
        batch.close()


def test_infinite_and_zero_temperature():
    need_gpu()
    _banner("T = inf / T = 0")
    w, mc, model, occ = make("c1", temperature=float("inf"))
    tr = mc.sweep(1, stats=True)
    assert tr["accepts"][0] == tr["diff_species"][0]
    mc.close()
    w, mc, model, occ = make("c1", temperature=0.0)
    tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
    acc = (tr["flags"] & 1).astype(bool)
    assert np.all(tr["dE"][acc] <= 0.0)
    mc.close()
