"""The double-lattice strategy (Algorithm 1 as written: sigma0/sigma1, all-site energies before
and after, zone reductions) against the zone strategy and the oracle, through the C ABI.

Bar: occupancy, energy cache and counters bit-identical to the zone strategy after every sweep
(same evaluator, same reduction order); FP32 against the FP64 oracle with the parity bar of the
zone strategy (decisions equal except within 1e-9 eV of the threshold)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import compare_sweep, make, need_gpu, trace_to_numpy

pytestmark = pytest.mark.gpu


def _banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _pair(prec, edges, temps, seed=5):
    import paper_2604_08250_amd as smc
    comps = [None, [0.4, 0.3, 0.2, 0.1], [0.1, 0.2, 0.3, 0.4]][:len(edges)]
    occ = np.concatenate([synth.random_occupancy(e, 4, c, seed=50 + r) for r, (e, c) in enumerate(zip(edges, comps))])
    params = synth.mlp_params(108, 128)
    out = []
    for strategy in ("zone", "double_lattice"):
        mc = smc.SwapMC([(e, e, e) for e in edges], temps, occ, params, n_species=4, feature=1, hidden=128,
                        precision=prec, seed=seed)
        mc.strategy = strategy
        assert mc.strategy == strategy
        out.append(mc)
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3", "fp8"])
def test_double_lattice_equals_zone(prec):
    need_gpu()
    _banner(f"double lattice vs zone {prec}")
    z, d = _pair(prec, [8, 9, 12], [600.0, 1500.0, 3000.0])
    for t in range(3):
        sz = trace_to_numpy(z.sweep(1, stats=True, trace=True))
        sd = trace_to_numpy(d.sweep(1, stats=True, trace=True))
        assert np.array_equal(z.occ.cpu().numpy(), d.occ.cpu().numpy()), f"sweep {t}: occupancy"
        assert np.array_equal(z.ecache.cpu().numpy(), d.ecache.cpu().numpy()), f"sweep {t}: energy cache"
        for k in ("attempts", "diff_species", "accepts", "rechecks"):
            assert np.array_equal(sz[k], sd[k]), (t, k)
        assert np.array_equal(sz["flags"], sd["flags"])
        assert np.array_equal(sz["dE_fast"], sd["dE_fast"])
    ez, rz = z.energy()
    ed, rd = d.energy()
    assert np.array_equal(ez, ed)
    assert np.allclose(rz, rd, rtol=0, atol=1e-8)
    # the double lattice's cache is still a from-scratch evaluation of the lattice
    assert np.array_equal(d.ecache.cpu().numpy(), d.site_energies(prec).cpu().numpy())
    z.close()
    d.close()


def test_double_lattice_fp32_matches_oracle():
    need_gpu()
    w, mc, model, occ = make("c2", cells=(8, 8, 8), temperature=800.0)
    mc.strategy = "double_lattice"
    _banner("double lattice fp32 vs oracle, 8^3")
    for t in range(4):
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        compare_sweep((8, 8, 8), model, occ, 800.0, w.seed, t, tr, mc.occ.cpu().numpy())
    es, er = mc.energy()
    assert es[0] == pytest.approx(oracle.total_energy((8, 8, 8), model, occ), abs=1e-9)
    mc.close()


def test_double_lattice_unsupported_configurations():
    need_gpu()
    import paper_2604_08250_amd as smc
    w, mc, _, _ = make("c1")  # counts model: per-lane path
    with pytest.raises(smc.SMCError):
        mc.strategy = "double_lattice"
    assert mc.strategy == "zone"
    mc.close()
    w, mc, _, _ = make("c2", cells=(8, 8, 8), precision="fp64")
    with pytest.raises(smc.SMCError):
        mc.strategy = "double_lattice"
    mc.close()
