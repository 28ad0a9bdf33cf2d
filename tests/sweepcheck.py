"""Colour-by-colour check of one GPU sweep on lattices too large for a whole oracle sweep.

A sweep of the GPU runs every colour (mini-step) in order.  Its trace gives, per trial site,
the decision, the dE of the sweep precision and whether the trial was re-decided in FP64.
Starting from the lattice before the sweep, each colour is checked on the lattice that the
GPU's own decisions of the earlier colours imply, then the GPU's accepted swaps of that
colour are applied on the host:

  - proposals (partner, threshold) come from the oracle, batched;
  - "full" colours: every different-species trial is re-evaluated by the library's FP64 probe
    (the evaluator that re-decides near-threshold trials) on that lattice.  The GPU decision
    must equal the FP64 one except within DECISION_BAND_EV of the threshold; trials the GPU
    re-decided in FP64 must carry exactly the probe's dE; trials it decided in the sweep
    precision must lie outside the guard band by that precision's own dE, and their error
    |dE_fast - dE_64| is collected (the evidence for the guard band);
  - sampled trials of every colour are evaluated by the oracle itself: its dE must equal the
    probe's within 1e-9 eV (which pins the probe to the oracle at this size), its decision
    must equal the GPU's outside the band, and the sweep precision's dE must lie within the
    precision's tolerance of it;
  - after the last colour the replayed lattice must equal the GPU's, bit for bit.
"""
from __future__ import annotations

import numpy as np

import oracle
from gpu_common import DECISION_BAND_EV


def colour_members(cells, c):
    """Trial sites of colour c in canonical order, for lattices whose edges are multiples of 4
    (link cells of 4 cells: colour = ((oz*4 + oy)*4 + ox)*2 + b)."""
    lx, ly, lz = cells
    assert lx % 4 == 0 and ly % 4 == 0 and lz % 4 == 0
    b = c % 2
    o = c // 2
    ox, oy, oz = o % 4, (o // 4) % 4, o // 16
    z = np.arange(oz, lz, 4, dtype=np.int64)
    y = np.arange(oy, ly, 4, dtype=np.int64)
    x = np.arange(ox, lx, 4, dtype=np.int64)
    s = ((z[:, None, None] * ly + y[None, :, None]) * lx + x[None, None, :]) * 2 + b
    return s.ravel()


def check_colour_rule(cells, rng, n=64):
    """The membership rule above against the oracle's schedule on random sites."""
    d = oracle._dims(cells)
    f = oracle.lib().or_colour_of
    dp = oracle._ptr(d, oracle.C.c_int32)
    for c in rng.choice(oracle.n_colours(cells), size=min(8, oracle.n_colours(cells)), replace=False):
        m = colour_members(cells, int(c))
        for s in rng.choice(m, size=min(n, m.size), replace=False):
            assert f(dp, int(s)) == c


class SweepStats:
    def __init__(self):
        self.full_trials = 0        # different-species trials checked against the FP64 probe
        self.max_err = 0.0          # max |dE_fast - dE_64| over them
        self.sum_sq = 0.0
        self.min_gap_fast = np.inf  # min |dE_fast - theta| of trials decided in the sweep precision
        self.tolerated = 0
        self.rechecked = 0
        self.sampled = 0
        self.max_probe_vs_oracle = 0.0

    @property
    def rms_err(self):
        return (self.sum_sq / max(self.full_trials, 1)) ** 0.5


def check_sweep(mc, probe, model, cells, T, seed, t, state, tr, full_colours, n_sample, rng, guard, de_tol,
                stats: SweepStats, log=None):
    """Check sweep t of `mc` (trace `tr`, numpy arrays) colour by colour starting from `state`
    (host copy of the lattice before the sweep; advanced in place to the lattice after it).
    probe: a second context on the same lattice shape whose occupancy tensor is overwritten
    with each colour's starting lattice; full_colours: colours probed trial by trial."""
    import torch

    flags, dE_fast, dE_dec = tr["flags"], tr["dE_fast"], tr["dE"]
    n_col = oracle.n_colours(cells)
    acc_total = diff_total = 0
    for c in range(n_col):
        m = colour_members(cells, c)
        _, part, theta = oracle.proposals(cells, seed, 0, t, T, m)
        si, sn = state[m], state[part]
        same = si == sn
        f = flags[m]
        assert np.array_equal((f & 2) != 0, same), f"sweep {t} colour {c}: same-species flags"
        acc = (f & 1) != 0
        assert not np.any(acc & same)
        d = ~same
        diff_total += int(d.sum())
        if c in full_colours:
            probe.occ.copy_(torch.from_numpy(state))
            md = m[d]
            pp, dE64 = probe.delta_e64(md, sweep=t)
            assert np.array_equal(pp, part[d]), f"sweep {t} colour {c}: partners of the library differ"
            th = theta[d]
            want = dE64 <= th
            gap = np.abs(dE64 - th)
            bad = (acc[d] != want) & (gap >= DECISION_BAND_EV)
            assert not bad.any(), (f"sweep {t} colour {c}: {int(bad.sum())} decisions differ from FP64, "
                                   f"first site {md[bad][0]} dE64 {dE64[bad][0]!r} theta {th[bad][0]!r} "
                                   f"dE_fast {dE_fast[md[bad][0]]!r}")
            stats.tolerated += int((acc[d] != want).sum())
            fp64 = (f[d] & 4) != 0
            stats.rechecked += int(fp64.sum())
            assert np.array_equal(dE_dec[md[fp64]], dE64[fp64]), f"sweep {t} colour {c}: re-decided dE"
            fast = ~fp64
            err = np.abs(dE_fast[md] - dE64)
            assert err.max(initial=0.0) < de_tol, f"sweep {t} colour {c}: max dE error {err.max()}"
            # a trial decided in the sweep precision lies outside the guard band by its own dE
            gap_fast = np.abs(dE_fast[md[fast]] - th[fast])
            assert np.all(gap_fast >= guard), f"sweep {t} colour {c}: fast decision inside the guard band"
            stats.min_gap_fast = min(stats.min_gap_fast, float(gap_fast.min(initial=np.inf)))
            stats.full_trials += int(d.sum())
            stats.max_err = max(stats.max_err, float(err.max(initial=0.0)))
            stats.sum_sq += float(np.sum(err * err))
        else:
            dE64 = None
        # sampled trials against the oracle itself
        cand = np.nonzero(d)[0]
        if cand.size and n_sample:
            for k in rng.choice(cand, size=min(n_sample, cand.size), replace=False):
                s = int(m[k])
                rec = oracle.trial(cells, model, state, T, seed, 0, t, s)
                assert rec["partner"] == part[k] and rec["theta"] == theta[k] and not rec["same"]
                if dE64 is not None:
                    j = int(np.searchsorted(m[d], s))
                    diff = abs(rec["dE"] - dE64[j])
                    assert diff < 1e-9, f"sweep {t} colour {c} site {s}: probe {dE64[j]!r} oracle {rec['dE']!r}"
                    stats.max_probe_vs_oracle = max(stats.max_probe_vs_oracle, diff)
                assert abs(dE_fast[s] - rec["dE"]) < de_tol
                if abs(rec["dE"] - rec["theta"]) >= DECISION_BAND_EV:
                    assert bool(acc[k]) == bool(rec["accept"]), f"sweep {t} colour {c} site {s}: decision"
                stats.sampled += 1
        # replay the GPU's accepted swaps of this colour
        a_sites, a_part = m[acc], part[acc]
        tmp = state[a_sites].copy()
        state[a_sites] = state[a_part]
        state[a_part] = tmp
        acc_total += int(acc.sum())
        if log is not None and (c % 32 == 31 or c == n_col - 1):
            log(f"sweep {t}: colours 0..{c} checked ({stats.full_trials} trials against FP64, "
                f"{stats.sampled} against the oracle)")
    return acc_total, diff_total
