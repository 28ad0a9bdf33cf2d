"""The qSRO model (Eq. 2) through the C ABI on the per-lane path, against the oracle.

Bar: site energies within 1e-12 (FP64) and 1e-6 eV (FP32) of the oracle; sweeps bit-exact with
the oracle under the same Philox stream, decisions equal except within 1e-9 eV of the
threshold (FP32 dE within 1e-6 eV), FP64 running totals equal the from-scratch total."""
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
    for t in range(8):
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        gocc = mc.occ.cpu().numpy()
        assert np.array_equal(np.bincount(gocc, minlength=S), counts0)
        compare_sweep(cells, model, occ, T, 7, t, tr, gocc, de_tol=1e-6)
    es, er = mc.energy()
    assert es[0] == pytest.approx(oracle.total_energy(cells, model, occ), abs=1e-9)
    assert abs(es[0] - er[0]) < 1e-6
    mc.close()
