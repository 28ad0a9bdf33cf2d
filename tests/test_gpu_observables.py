"""Warren-Cowley short-range order and temperature changes through the C ABI.

Bar: alpha equal to the oracle's (integer pair counts, the same FP64 formula) on every replica
of a mixed batch, including a species that is absent; after a temperature change, sweeps equal
the oracle's sweeps at the new temperature (decisions equal except within the recheck band of
the threshold), on the per-launch path and on replays of the captured sweep."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import compare_sweep, make, need_gpu, trace_to_numpy

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _slices(mc):
    out, s0 = [], 0
    for c in mc.cells:
        n = 2 * int(np.prod(c))
        out.append((tuple(int(x) for x in c), slice(s0, s0 + n)))
        s0 += n
    return out


@pytest.mark.parametrize("model", ["mlp", "qsro"])
def test_warren_cowley_matches_oracle(model):
    need_gpu()
    import paper_2604_08250_amd as smc
    S = 4 if model == "mlp" else 5
    edges = [(4, 4, 4), (6, 5, 7), (9, 9, 9)]
    occ = [synth.random_occupancy(edges[0], S, None, seed=61),
           synth.random_occupancy(edges[1], S, None, seed=62),
           (np.arange(oracle.n_sites(edges[2])) % 2).astype(np.uint8)]  # B2 order, species 2.. absent
    occ = np.concatenate(occ)
    if model == "mlp":
        params, feature, hidden = synth.mlp_params(108, 128), 1, 128
    else:
        params, feature, hidden = synth.qsro_params(n_species=S), smc.SMC_FEAT_QSRO_S123, 0
    _banner(f"warren-cowley {model} S={S}")
    mc = smc.SwapMC(edges, [700.0, 1500.0, 400.0], occ, params, n_species=S, feature=feature,
                    hidden=hidden, precision="fp32", seed=8)
    for sweeps in (0, 3):
        if sweeps:
            mc.sweep(sweeps)
        now = mc.occ.cpu().numpy()
        for r, (cells, sl) in enumerate(_slices(mc)):
            want = oracle.warren_cowley(cells, now[sl], S)
            got = mc.warren_cowley(r)
            np.testing.assert_allclose(got, want, rtol=0, atol=1e-14, err_msg=f"replica {r} after {sweeps}")
    # B2 before any sweep: nearest neighbours all unlike, second shell all like
    a = oracle.warren_cowley(edges[2], occ[_slices(mc)[2][1]], S)
    assert a[0, 0, 1] == pytest.approx(-1.0) and a[1, 0, 0] == pytest.approx(-1.0)
    with pytest.raises(smc.SMCError):
        smc.smc_warren_cowley(mc.ctx, 3, S)
    mc.close()


@pytest.mark.parametrize("graph", [False, True])
def test_temperature_change_follows_oracle(graph):
    need_gpu()
    import paper_2604_08250_amd as smc
    cells = (8, 8, 8)
    w, mc, model, occ = make("c2", cells=cells, temperature=800.0)
    if graph:
        mc.use_graph(True)
    schedule = [800.0, 800.0, 2500.0, 2500.0, 300.0, float("inf")]
    _banner(f"temperature schedule graph={graph}")
    for t, T in enumerate(schedule):
        if t and T != schedule[t - 1]:
            mc.set_temperatures(T)
        if graph:
            mc.sweep(1)
            st, _ = oracle.sweep(cells, model, occ, T, w.seed, 0, t, trace=True, nthreads=8)
            assert np.array_equal(mc.occ.cpu().numpy(), occ), f"sweep {t} at {T} K"
        else:
            tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
            compare_sweep(cells, model, occ, T, w.seed, t, tr, mc.occ.cpu().numpy())
    assert mc.temperatures[0] == float("inf")
    es, er = mc.energy()
    assert es[0] == pytest.approx(oracle.total_energy(cells, model, occ), abs=1e-9)
    for bad in (-1.0, float("nan")):
        with pytest.raises(smc.SMCError):
            mc.set_temperatures(bad)
    mc.close()


def test_anneal_helper_equals_manual_schedule():
    need_gpu()
    a = make("c2", cells=(8, 8, 8), temperature=3000.0)[1]
    b = make("c2", cells=(8, 8, 8), temperature=3000.0)[1]
    _banner("anneal helper")
    a.anneal([3000.0, 1500.0, 600.0], 2)
    for T in (3000.0, 1500.0, 600.0):
        b.set_temperatures(T)
        b.sweep(1)
        b.sweep(1)
    assert np.array_equal(a.occ.cpu().numpy(), b.occ.cpu().numpy())
    assert a.sweep_index == b.sweep_index == 6
    a.close()
    b.close()


def test_observable_error_of_each_precision():
    """Chains of every precision from one start and Philox stream (32^3 cells, T = 800 K, 120
    sweeps, samples every 2 after 40): FP32 and split BF16 must be the FP64-mode chain itself;
    plain BF16 and FP8 follow their own chains, and their E per atom and Warren-Cowley alpha of
    shells 1-2 (Eq. (3) pair fractions averaged over the lattice) must stay within loose bounds
    of the FP64 chain's (printed: the observable error of each precision)."""
    need_gpu()
    res, final = {}, {}
    for p in ("fp64", "fp32", "bf16x3", "bf16", "fp8"):
        w, mc, model, occ = make("c2", precision=p, cells=(32, 32, 32))
        n = occ.size
        E, al = [], []
        for s in range(60):
            mc.sweep(2)
            if s >= 20:
                E.append(mc.energy()[0][0] / n)
                al.append(mc.warren_cowley()[:2])
        final[p] = mc.occ.cpu().numpy()
        res[p] = (np.mean(E), np.mean(al, axis=0))
        mc.close()
    for p in ("fp32", "bf16x3"):
        assert np.array_equal(final[p], final["fp64"]), f"{p} chain left the FP64 chain"
    for p, (tol_e, tol_a) in {"bf16": (1e-4, 0.02), "fp8": (1e-3, 0.05)}.items():
        dE = res[p][0] - res["fp64"][0]
        da = float(np.abs(res[p][1] - res["fp64"][1]).max())
        _banner(f"{p}: E/atom {res[p][0]:.6f} vs FP64 {res['fp64'][0]:.6f} eV (diff {dE:+.2e}), max |d alpha| {da:.4f}")
        assert abs(dE) < tol_e and da < tol_a
