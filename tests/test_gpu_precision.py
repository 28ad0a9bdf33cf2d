"""Matrix-core evaluators and low-precision sweeps.

* Each precision's site energies match a CPU emulation of that precision's model (this
  catches packing, operand-layout and scale mistakes) and the FP64 oracle within the
  precision's own error.
* FP32 and split-BF16 sweeps are bit-exact with the oracle (decisions near the threshold
  are re-decided in FP64 inside the guard band).
* BF16 and FP8 sweeps keep composition, keep the energy cache equal to a from-scratch
  evaluation with the same evaluator, and report their dE error against FP64.
"""
import numpy as np
import pytest

import oracle
from emulate import energies as emulate_energies
from gpu_common import compare_sweep, make, need_gpu, trace_to_numpy

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16x3", "bf16", "fp8"]


def _banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _features(cells, occ, n):
    X = np.stack([oracle.features(cells, oracle.FEAT_ONEHOT_S123, occ, j) for j in range(n)])
    return X


@pytest.mark.parametrize("prec", PRECS)
def test_site_energies_match_emulation_and_oracle(prec):
    need_gpu()
    cells = (8, 12, 16)
    w, mc, model, occ = make("c2", precision=prec, cells=cells, n_species=5)
    e_gpu = mc.site_energies(prec).cpu().numpy().astype(np.float64)
    n = 1500
    X = _features(cells, occ, n)
    e_emu = emulate_energies(w.params(), X, prec)
    e64 = oracle.all_site_energies(cells, model, occ)[:n]
    d_emu = np.abs(e_gpu[:n] - e_emu)
    d_64 = np.abs(e_gpu[:n] - e64)
    d_emu64 = np.abs(e_emu - e64)
    _banner(f"{prec}: |gpu-emu| max {d_emu.max():.3e} rms {np.sqrt((d_emu**2).mean()):.3e}; "
            f"|gpu-fp64| max {d_64.max():.3e}; |emu-fp64| max {d_emu64.max():.3e}")
    # the energy cache was filled by the same evaluator
    assert np.array_equal(mc.ecache.cpu().numpy(), e_gpu.astype(np.float32))
    if prec == "fp32":
        assert d_emu.max() < 2e-6 and d_64.max() < 5e-6
    elif prec == "bf16x3":
        assert d_emu.max() < 2e-5 and d_64.max() < 1e-4
    else:
        # activation roundings may flip at ties between GPU and emulation: the disagreement
        # must stay far below the precision's own error
        assert np.sqrt((d_emu**2).mean()) < 0.1 * np.sqrt((d_emu64**2).mean())
        assert np.median(d_emu) < 0.05 * np.median(d_emu64) + 1e-6
    mc.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_one_hot_sweeps_bit_exact(prec):
    need_gpu()
    cells = (8, 8, 8)
    _banner(f"one-hot 8^3 {prec}")
    w, mc, model, occ = make("c2", precision=prec, cells=cells, temperature=800.0)
    worst = 0.0
    for t in range(4):
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        n_tol, otr = compare_sweep(cells, model, occ, 800.0, w.seed, t, tr, mc.occ.cpu().numpy(),
                                   de_tol=1e-5 if prec == "fp32" else 1e-4)
        d = otr["same"] == 0
        worst = max(worst, float(np.abs(tr["dE_fast"][d] - otr["dE"][d]).max()))
    _banner(f"{prec}: max |dE_fast - dE_fp64| = {worst:.3e}, guard {'1e-5' if prec == 'fp32' else '1e-4'}")
    assert worst < (2.5e-5 if prec == "bf16x3" else 2e-6)  # guard / 4 (bf16x3), guard / 5 (fp32)
    if prec == "fp64":
        # every different-species trial was decided by the FP64 evaluator
        flags = tr["flags"]
        assert np.all((flags & 4).astype(bool) == ~(flags & 2).astype(bool))
    else:
        assert np.array_equal(mc.ecache.cpu().numpy(), mc.site_energies(prec).cpu().numpy())
    mc.close()


def test_fp64_probe_matches_oracle():
    """smc_delta_e64 (the FP64 evaluator of the re-decision path) against the oracle."""
    need_gpu()
    cells = (12, 8, 16)
    w, mc, model, occ = make("c2", precision="bf16", cells=cells, n_species=5)
    sites = np.arange(0, occ.size, 7)
    partner, dE = mc.delta_e64(sites, sweep=3)
    for s, p, e in zip(sites, partner, dE):
        rec = oracle.trial(cells, model, occ, 800.0, w.seed, 0, 3, int(s))
        assert p == rec["partner"]
        assert abs(e - rec["dE"]) < 1e-11
    assert np.array_equal(mc.occ.cpu().numpy(), occ)  # nothing changed
    mc.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_low_precision_chain_consistency(prec):
    need_gpu()
    cells = (16, 16, 16)
    _banner(f"low precision chain {prec}")
    w, mc, model, occ = make("c2", precision=prec, cells=cells, temperature=800.0)
    counts0 = np.bincount(occ, minlength=4)
    errs = []
    for t in range(3):
        before = mc.occ.cpu().numpy().copy()
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        after = mc.occ.cpu().numpy()
        assert np.array_equal(np.bincount(after, minlength=4), counts0)
        assert tr["attempts"][0] == occ.size
        # dE error of sampled trials of colour 0 (decided on the pre-sweep lattice)
        col0 = [s for s in range(0, occ.size, 2) if oracle.lib().or_colour_of(
            oracle._ptr(oracle._dims(cells), oracle.C.c_int32), s) == 0][:24]
        for s in col0:
            rec = oracle.trial(cells, model, before, 800.0, w.seed, 0, t, s)
            if not rec["same"]:
                errs.append(tr["dE_fast"][s] - rec["dE"])
    errs = np.array(errs)
    _banner(f"{prec}: dE error vs FP64 over {errs.size} trials: rms {np.sqrt((errs**2).mean()):.3e} "
            f"max {np.abs(errs).max():.3e}")
    assert np.array_equal(mc.ecache.cpu().numpy(), mc.site_energies(prec).cpu().numpy())
    assert np.sqrt((errs**2).mean()) < (0.02 if prec == "bf16" else 0.2)
    es, er = mc.energy()
    _banner(f"{prec}: E_running - E_scratch = {er[0] - es[0]:.3e} eV over {occ.size} sites")
    mc.close()
