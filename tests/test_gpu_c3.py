"""The headline lattice (BCC 256^3 cells, 33,554,432 sites, five species, T = 600 K, the
108 -> 128 -> 128 -> 1 one-hot MLP) and the 64^3 lattice, checked colour by colour through
the C ABI, in the launch configuration the benchmark times (graph-free per-launch sweeps with
traces; the same kernels and grid as graph replays, which are bit-identical by test).

Bar (Algorithm 1, Sec. III-A; one trial per site per sweep, Sec. V-A):
  - every different-species trial of the probed colours decided as the FP64 evaluator decides
    it, except within 1e-9 eV of the threshold; trials re-decided in FP64 carry its exact dE;
  - the FP64 evaluator equal to the oracle within 1e-9 eV on sampled trials of every colour,
    and the GPU decisions equal to the oracle's there;
  - the sweep precision's dE within 1e-5 eV (FP32) or 1e-4 eV (split BF16) of FP64, and
    within the guard band on every probed trial (recorded: the evidence for the band);
  - the lattice after each sweep equal to the replay of the GPU's decisions, the counters equal
    to the replay's, the energy cache equal to a from-scratch evaluation bit for bit and the
    running total equal to the FP64 total within the accumulated dE error.
"""
import numpy as np
import pytest

import oracle
from gpu_common import make, need_gpu, trace_to_numpy
from sweepcheck import SweepStats, check_colour_rule, check_sweep

pytestmark = pytest.mark.gpu

GUARD = {"fp32": 1e-5, "bf16x3": 1e-4}
DE_TOL = {"fp32": 1e-5, "bf16x3": 1e-4}


def _banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def _run(name, precision, n_sweeps, full, n_sample):
    import paper_2604_08250_amd as smc
    need_gpu()
    w, mc, model, occ = make(name, precision=precision)
    cells, T = w.cells[0], w.temperatures[0]
    rng = np.random.default_rng(12)
    check_colour_rule(cells, rng)
    probe = smc.SwapMC(w.cells, w.temperatures, occ, w.params(), n_species=w.n_species, feature=w.feature,
                       hidden=w.hidden, precision="fp32", seed=w.seed)
    state = occ.copy()
    st = SweepStats()
    accepts = 0
    for t in range(n_sweeps):
        _banner(f"{name} {precision}: sweep {t}")
        tr = trace_to_numpy(mc.sweep(1, stats=True, trace=True))
        acc, diff = check_sweep(mc, probe, model, cells, T, w.seed, t, state, tr, full(t), n_sample, rng,
                                GUARD[precision], DE_TOL[precision], st, log=_banner)
        assert np.array_equal(state, mc.occ.cpu().numpy()), f"lattice after sweep {t} differs from the replay"
        assert tr["attempts"][0] == state.size and tr["diff_species"][0] == diff and tr["accepts"][0] == acc
        accepts += acc
    _banner(f"{name} {precision}: {st.full_trials} trials against FP64: max |dE err| {st.max_err:.3e} eV, "
            f"RMS {st.rms_err:.3e}, min |dE_fast - theta| of fast decisions {st.min_gap_fast:.3e}, "
            f"re-decided {st.rechecked}, tolerated {st.tolerated}; {st.sampled} oracle trials, "
            f"max |probe - oracle| {st.max_probe_vs_oracle:.3e}")
    # the recorded evidence for the guard band: the largest error stays below a quarter of it
    assert st.max_err < GUARD[precision] / 4
    assert np.array_equal(mc.ecache.cpu().numpy(), mc.site_energies(precision).cpu().numpy())
    es, er = mc.energy()
    assert abs(es[0] - er[0]) <= 10.0 * max(st.max_err, 1e-9) * np.sqrt(accepts) + 1e-9 * abs(es[0])
    mc.close()
    probe.close()
    return st


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_c3_headline_every_trial_of_sweep0_against_fp64(precision):
    """256^3: every trial of every colour of the first sweep against the FP64 evaluator (26.8 M
    different-species trials), the first 16 colours of the second in full and the rest sampled;
    three oracle trials per colour."""
    _run("c3", precision, 2, lambda t: set(range(128)) if t == 0 else set(range(16)), 3)


def test_c2_ten_sweeps_every_trial_against_fp64():
    """64^3 FP32: ten sweeps, every trial against the FP64 evaluator, three oracle trials per
    colour and sweep."""
    _run("c2", "fp32", 10, lambda t: set(range(128)), 3)


def test_c2_fp32_and_split_bf16_chains_equal_fp64_mode():
    """64^3: the FP64 mode decides every trial with the FP64 evaluator; the FP32 and split-BF16
    modes decide outside their guard bands in their own precision and re-decide inside them
    with the same FP64 evaluator.  Their chains must therefore be the FP64 chain, bit for bit,
    sweep after sweep (60 sweeps, 3.1e7 trials each)."""
    need_gpu()
    ctx = {p: make("c2", precision=p)[1] for p in ("fp64", "fp32", "bf16x3")}
    for blk in range(6):
        for mc in ctx.values():
            mc.sweep(10)
        ref = ctx["fp64"].occ.cpu().numpy()
        for p in ("fp32", "bf16x3"):
            assert np.array_equal(ctx[p].occ.cpu().numpy(), ref), f"{p} chain left the FP64 chain by sweep {10 * blk + 10}"
        _banner(f"c2 chains equal after {10 * blk + 10} sweeps")
    cnt = {p: mc.counters() for p, mc in ctx.items()}
    assert np.array_equal(cnt["fp32"][:3], cnt["fp64"][:3]) and np.array_equal(cnt["bf16x3"][:3], cnt["fp64"][:3])
    _banner(f"re-decided in FP64: fp32 {int(cnt['fp32'][3][0])}, bf16x3 {int(cnt['bf16x3'][3][0])} "
            f"of {int(cnt['fp64'][1][0])} different-species trials")
    for mc in ctx.values():
        mc.close()
