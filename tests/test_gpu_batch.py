"""Batched replicas, graph-captured sweeps and kernel variants, through the C ABI.

Bar: graph replays and every kernel variant reproduce the per-launch sweep bit for bit
(occupancy, energy cache, counters, running energies); the autotuner leaves the caller's state
untouched; the full 96-replica workload in BF16 agrees with the FP64 oracle on sampled trials
of every colour of several replicas, decided on the state the GPU's own decisions imply.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import need_gpu, trace_to_numpy

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _uneven(prec, seed=5, graph=True, variant=None, edges=(8, 9, 12, 20), temps=(500.0, 1200.0, 3000.0, 800.0)):
    import paper_2604_08250_amd as smc
    comps = [None, [0.4, 0.3, 0.2, 0.1], [0.1, 0.2, 0.3, 0.4], [0.25, 0.25, 0.3, 0.2], [0.3, 0.2, 0.2, 0.3]]
    comps = comps[:len(edges)]
    assert len(comps) == len(edges) == len(temps)
    occ = np.concatenate([synth.random_occupancy(e, 4, c, seed=10 + r) for r, (e, c) in enumerate(zip(edges, comps))])
    params = synth.mlp_params(108, 128)
    mc = smc.SwapMC([(e, e, e) for e in edges], list(temps)[:len(edges)], occ, params, n_species=4, feature=1,
                    hidden=128, precision=prec, seed=seed)
    mc.use_graph(graph)
    if variant is not None:
        mc.variant = variant
    return mc


def _state(mc):
    es, er = mc.energy()
    return (mc.occ.cpu().numpy().copy(), mc.ecache.cpu().numpy().copy(), mc.counters(), er, mc.sweep_index)


def _assert_same_state(a, b, what):
    assert np.array_equal(a[0], b[0]), f"{what}: occupancy"
    assert np.array_equal(a[1], b[1]), f"{what}: energy cache"
    assert np.array_equal(a[2], b[2]), f"{what}: counters"
    assert np.array_equal(a[3], b[3]), f"{what}: running energies"
    assert a[4] == b[4], f"{what}: sweep index"


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp8"])
def test_graph_replay_equals_per_launch(prec):
    """Replays of the captured sweep, with eager work and synchronisations between them, give
    the per-launch sweep's results after every replay."""
    need_gpu()
    _banner(f"graph vs per-launch {prec}")
    g = _uneven(prec, graph=True)
    e = _uneven(prec, graph=False)
    for t in range(5):
        g.sweep(1)
        e.sweep(1)
        # eager work between replays on the same stream
        _ = g.site_energies("fp32")
        _ = e.site_energies("fp32")
        _assert_same_state(_state(g), _state(e), f"sweep {t}")
    # several sweeps per call, then a stats call (per-launch) in the middle of graph replays
    g.sweep(3)
    e.sweep(3)
    sg = g.sweep(1, stats=True)
    se = e.sweep(1, stats=True)
    for k in ("attempts", "diff_species", "accepts", "rechecks"):
        assert np.array_equal(sg[k], se[k]), k
    g.sweep(2)
    e.sweep(2)
    _assert_same_state(_state(g), _state(e), "after mixed calls")
    # the occupancy evolved and every replica conserved its composition
    g.close()
    e.close()


def test_variants_bit_identical():
    need_gpu()
    ref = None
    for v in range(4):
        _banner(f"variant {v}")
        mc = _uneven("bf16", variant=v, edges=(8, 9, 12, 20, 32), temps=(500.0, 1200.0, 3000.0, 800.0, 650.0))
        assert mc.variant == v
        mc.sweep(3)
        st = _state(mc)
        if ref is None:
            ref = st
        else:
            _assert_same_state(st, ref, f"variant {v}")
        mc.close()


def test_autotune_restores_state_and_uses_cache(tmp_path):
    need_gpu()
    _banner("autotune")
    cache = str(tmp_path / "tune.jsonl")
    a = _uneven("bf16")
    b = _uneven("bf16")
    a.sweep(2)
    b.sweep(2)
    before = _state(a)
    v, ms = a.autotune(cache)
    _banner(f"chosen {v}, ms per variant {ms}")
    assert 0 <= v < 4 and a.variant == v
    assert np.all(ms > 0.0)
    _assert_same_state(_state(a), before, "after autotune")
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and f'"variant": {v}' in lines[0]
    # a second context with the same shapes reads the cache without timing
    v2, ms2 = b.autotune(cache)
    assert v2 == v and np.all(ms2 == 0.0)
    assert len(open(cache).read().splitlines()) == 1
    # the tuned context continues exactly like an untuned one
    a.sweep(3)
    b.variant = 0
    b.sweep(3)
    _assert_same_state(_state(a), _state(b), "tuned vs variant 0")
    a.close()
    b.close()


def test_c4_batched_sampled():
    """The 96-replica workload (cube edges 16..96, random compositions, 300..3000 K) in BF16:
    one graph-replayed sweep equals the per-launch sweep bit for bit; on the per-launch trace,
    sampled trials of every colour of four replicas are re-decided by the oracle in FP64 on
    the state that the GPU's earlier decisions imply."""
    torch = need_gpu()
    import paper_2604_08250_amd as smc
    w = synth.workload("c4")
    occ0 = w.occupancy()
    params = w.params()
    sizes = [2 * int(np.prod(c)) for c in w.cells]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    _banner(f"c4: {len(w.cells)} replicas, {offs[-1]} sites")
    mcs = []
    for graph in (True, False):
        mc = smc.SwapMC(w.cells, w.temperatures, occ0, params, n_species=w.n_species, feature=w.feature,
                        hidden=w.hidden, precision="bf16", seed=w.seed)
        mc.use_graph(graph)
        mcs.append(mc)
    g, e = mcs
    g.sweep(1)
    tr = trace_to_numpy(e.sweep(1, stats=True, trace=True))
    gocc = g.occ.cpu().numpy()
    eocc = e.occ.cpu().numpy()
    assert np.array_equal(gocc, eocc)
    assert np.array_equal(g.ecache.cpu().numpy(), e.ecache.cpu().numpy())
    assert np.array_equal(g.counters(), e.counters())
    g.close()
    del g
    torch.cuda.empty_cache()
    assert np.array_equal(tr["attempts"], np.asarray(sizes, dtype=np.uint64))
    for r in range(len(sizes)):
        a, b = offs[r], offs[r + 1]
        assert np.array_equal(np.bincount(eocc[a:b], minlength=4), np.bincount(occ0[a:b], minlength=4))
    model = oracle.MLP(w.feature, w.hidden, params)
    order = np.argsort(sizes)
    picks = [int(order[0]), int(order[1]), int(order[len(order) // 2]), int(order[-1])]
    rng = np.random.default_rng(1)
    errs = []
    for r in picks:
        cells, T = w.cells[r], w.temperatures[r]
        a, b = offs[r], offs[r + 1]
        occ = occ0[a:b].copy()
        flags = tr["flags"][a:b]
        dE = tr["dE"][a:b]
        dEf = tr["dE_fast"][a:b]
        col = oracle.colours(cells)
        nc = oracle.n_colours(cells)
        _banner(f"c4 replica {r}: cells {cells}, T {T:.0f} K, {nc} colours")
        for c in range(nc):
            members = np.nonzero(col == c)[0]
            for s in rng.choice(members, size=min(2, members.size), replace=False):
                rec = oracle.trial(cells, model, occ, T, w.seed, r, 0, int(s))
                assert bool(flags[s] & 2) == bool(rec["same"])
                if rec["same"]:
                    continue
                errs.append(dEf[s] - rec["dE"])
                if flags[s] & 4:  # re-decided in FP64: the oracle's decision
                    assert abs(dE[s] - rec["dE"]) < 1e-9
                    if abs(rec["dE"] - rec["theta"]) >= 1e-9:
                        assert bool(flags[s] & 1) == bool(rec["accept"])
                else:  # decided in BF16 outside the guard band
                    assert bool(flags[s] & 1) == bool(dEf[s] <= rec["theta"])
                    assert abs(dEf[s] - rec["theta"]) >= 1e-5 * (1 - 1e-12)
            acc = members[(flags[members] & 1).astype(bool)]
            for s in acc:
                d, _ = oracle.propose(w.seed, int(s), 0, r)
                n = oracle.neighbor(cells, int(s), d)
                occ[s], occ[n] = occ[n], occ[s]
        assert np.array_equal(occ, eocc[a:b]), f"replica {r}: replayed decisions"
    errs = np.asarray(errs)
    _banner(f"c4 bf16 dE error vs FP64 over {errs.size} trials: rms {np.sqrt((errs ** 2).mean()):.3e} "
            f"max {np.abs(errs).max():.3e}")
    assert np.sqrt((errs ** 2).mean()) < 0.02
    e.close()


def test_many_replicas_counters_and_parity():
    """70 replicas (more counters than one block of threads): every replica's counters are
    consistent from the first sweep, and sampled replicas match the oracle bit for bit."""
    need_gpu()
    import paper_2604_08250_amd as smc
    R = 70
    edges = [4 + (r % 3) for r in range(R)]
    temps = [300.0 + 40.0 * r for r in range(R)]
    params = synth.mlp_params(108, 128)
    occs = [synth.random_occupancy(e, 4, None, seed=200 + r) for r, e in enumerate(edges)]
    cells = [(e, e, e) for e in edges]
    _banner(f"{R} replicas")
    mc = smc.SwapMC(cells, temps, np.concatenate(occs), params, n_species=4, feature=1, hidden=128,
                    precision="fp32", seed=9)
    st = mc.sweep(2, stats=True)
    sizes = np.array([o.size for o in occs], dtype=np.uint64)
    assert np.array_equal(st["attempts"], 2 * sizes)
    assert np.all(st["diff_species"] <= st["attempts"])
    assert np.all(st["accepts"] <= st["diff_species"])
    assert np.all(st["rechecks"] <= st["diff_species"])
    cnt = mc.counters()
    assert np.array_equal(cnt[0], st["attempts"]) and np.array_equal(cnt[2], st["accepts"])
    got = mc.occ.cpu().numpy()
    model = oracle.MLP(1, 128, params)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    for r in (0, 64, 69):
        ref = occs[r].copy()
        for t in range(2):
            oracle.sweep(cells[r], model, ref, temps[r], 9, r, t, nthreads=8)
        assert np.array_equal(got[offs[r]:offs[r + 1]], ref), f"replica {r}"
    mc.close()
