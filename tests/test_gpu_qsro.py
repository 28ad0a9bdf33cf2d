"""The qSRO model (Eq. 2) through the C ABI, against the oracle: FP32 sweeps run in the tiled
colour kernel (regions staged in LDS, per-lane qSRO evaluation, FP64 re-decision of the queue),
FP64 sweeps on the per-lane path.

Bar: site energies within 1e-12 (FP64) and 1e-6 eV (FP32) of the oracle; sweeps bit-exact with
the oracle under the same Philox stream, decisions equal except within 1e-9 eV of the
threshold (FP32 dE within 1e-6 eV); running totals equal the from-scratch total up to the
random walk of the per-trial dE error."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import compare_sweep, need_gpu, trace_to_numpy

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _make(cells, n_species, precision, T=1000.0, seed=7):
    import paper_2604_08250_amd as smc
    P = synth.qsro_params(n_species)
    occ = synth.random_occupancy(cells, n_species, None, seed=3)
    mc = smc.SwapMC([cells], [T], occ, P, n_species=n_species, feature=2, hidden=0, precision=precision, seed=seed)
    return mc, oracle.QSRO(P), occ.copy()


def test_qsro_site_energies():
    need_gpu()
    for cells, S in [((8, 8, 8), 4), ((9, 10, 13), 5)]:
        _banner(f"qSRO site energies {cells} S={S}")
        mc, model, occ = _make(cells, S, "fp32")
        want = oracle.all_site_energies(cells, model, occ)
        assert np.max(np.abs(mc.site_energies("fp64").cpu().numpy() - want)) < 1e-12
        assert np.max(np.abs(mc.site_energies("fp32").cpu().numpy() - want)) < 1e-6
        es, er = mc.energy()
        assert es[0] == pytest.approx(want.sum(), abs=1e-9)
        mc.close()


@pytest.mark.parametrize("precision,cells,S", [("fp32", (8, 8, 8), 4), ("fp64", (8, 8, 8), 4),
                                               ("fp32", (9, 10, 13), 5)])
def test_qsro_sweeps_bit_exact(precision, cells, S):
    need_gpu()
    T = 700.0
    mc, model, occ = _make(cells, S, precision, T=T)
    _banner(f"qSRO {precision} {cells} S={S}")
    counts0 = np.bincount(occ, minlength=S)
    accepts = 0
    max_err = 0.0
    for t in range(8):
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        gocc = mc.occ.cpu().numpy()
        assert np.array_equal(np.bincount(gocc, minlength=S), counts0)
        _, otr = compare_sweep(cells, model, occ, T, 7, t, tr, gocc, de_tol=1e-6)
        accepts += int(tr["accepts"][0])
        d = otr["same"] == 0
        max_err = max(max_err, float(np.abs(tr["dE"][d] - otr["dE"][d]).max(initial=0.0)))
    es, er = mc.energy()
    assert es[0] == pytest.approx(oracle.total_energy(cells, model, occ), abs=1e-9)
    # the running total adds each accepted swap's deciding dE, so it drifts from the from-scratch
    # total like a random walk of the per-trial dE error (exactly equal in FP64)
    assert abs(es[0] - er[0]) <= 10.0 * max_err * np.sqrt(max(accepts, 1)) + 1e-9 * abs(es[0])
    mc.close()


@pytest.mark.parametrize("model_name", ["qsro", "counts"])
def test_batch_matches_oracle_per_replica(model_name):
    """Replicas of different shapes and temperatures in one context, one launch per colour over
    every replica that has it (qSRO: the tiled colour kernel, groups of link cells mapped to
    their replica; counts model: the per-lane path, each block serving one replica): every
    replica equals the oracle's own sweeps of that replica."""
    need_gpu()
    import paper_2604_08250_amd as smc
    qsro = model_name == "qsro"
    cells = [(4, 4, 4), (6, 5, 7), (9, 9, 9), (5, 5, 5)]
    temps = [400.0, 900.0, 1500.0, 2500.0]
    S = 5 if qsro else 4
    P = synth.qsro_params(S) if qsro else synth.mlp_params(12, 64)
    occs = [synth.random_occupancy(c, S, None, seed=300 + r) for r, c in enumerate(cells)]
    _banner(f"batch {model_name}: {len(cells)} replicas")
    mc = smc.SwapMC(cells, temps, np.concatenate(occs), P, n_species=S, feature=2 if qsro else 0,
                    hidden=0 if qsro else 64, precision="fp32", seed=11)
    st = mc.sweep(3, stats=True)
    sizes = np.array([o.size for o in occs], dtype=np.uint64)
    assert np.array_equal(st["attempts"], 3 * sizes)
    got = mc.occ.cpu().numpy()
    model = oracle.QSRO(P) if qsro else oracle.MLP(0, 64, P)
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    for r in range(len(cells)):
        ref = occs[r].copy()
        for t in range(3):
            oracle.sweep(cells[r], model, ref, temps[r], 11, r, t, nthreads=8)
        assert np.array_equal(got[offs[r]:offs[r + 1]], ref), f"replica {r}"
    mc.close()


def test_qsro_graph_replay_equals_per_launch():
    """FP32 qSRO sweeps run in the captured colour-kernel path: replays of the captured sweep
    over uneven replicas, with eager work between them, equal the per-launch sweeps after every
    replay (occupancy, energy cache, counters, running energies)."""
    need_gpu()
    import paper_2604_08250_amd as smc
    cells = [(8, 8, 8), (9, 10, 13), (12, 12, 12)]
    temps = [600.0, 1200.0, 2500.0]
    P = synth.qsro_params(5)
    occ = np.concatenate([synth.random_occupancy(c, 5, None, seed=40 + r) for r, c in enumerate(cells)])
    _banner("qSRO graph vs per-launch")
    runs = []
    for graph in (True, False):
        mc = smc.SwapMC(cells, temps, occ, P, n_species=5, feature=2, hidden=0, precision="fp32", seed=13)
        mc.use_graph(graph)
        runs.append(mc)
    g, e = runs
    for t in range(5):
        g.sweep(1)
        e.sweep(1)
        _ = g.site_energies("fp64")  # eager work between replays
        sg, se = g.energy(), e.energy()
        assert np.array_equal(g.occ.cpu().numpy(), e.occ.cpu().numpy()), f"sweep {t}: occupancy"
        assert np.array_equal(g.ecache.cpu().numpy(), e.ecache.cpu().numpy()), f"sweep {t}: energy cache"
        assert np.array_equal(g.counters(), e.counters()), f"sweep {t}: counters"
        assert np.array_equal(sg[1], se[1]), f"sweep {t}: running energies"
    g.close()
    e.close()
