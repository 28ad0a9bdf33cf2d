"""Pins of the oracle's qSRO local energy (Eq. 2) against closed forms worked out by hand on
ordered structures, a single substitution, the zone invariant (dE equals the total-energy
difference) and exact Boltzmann stationarity on the 16-site lattice."""
import math

import numpy as np
import pytest

import oracle
import synth

KB = oracle.KB_EV_PER_K
Z = {1: 8, 2: 6, 3: 12}


def _parts(P):
    P = np.asarray(P, dtype=np.float64)
    return P[:75].reshape(3, 5, 5), P[75:90].reshape(3, 5), P[90], P[91]


def test_pure_element_closed_form():
    """Every pair is like: pi_m^{00} = 1, so E = C + sum_m W_m^0 + lambda sum W^2 per site."""
    P = synth.qsro_params()
    V, W, lam, C = _parts(P)
    cells = (4, 4, 4)
    occ = np.zeros(oracle.n_sites(cells), dtype=np.uint8)
    want = C + W[:, 0].sum() + lam * (W ** 2).sum()
    assert oracle.total_energy(cells, oracle.QSRO(P), occ) == pytest.approx(occ.size * want, abs=1e-12)


def test_b2_closed_form():
    """B2 (species 0 on corners, 1 on body centres): shell 1 is all unlike (pi^{10} = 1),
    shells 2 and 3 all like."""
    P = synth.qsro_params()
    V, W, lam, C = _parts(P)
    cells = (4, 4, 4)
    N = oracle.n_sites(cells)
    occ = (np.arange(N) % 2).astype(np.uint8)
    reg = lam * (W ** 2).sum()
    e0 = C + V[0, 1, 0] + W[1, 0] + W[2, 0] + reg
    e1 = C + V[0, 1, 0] + W[1, 1] + W[2, 1] + reg
    m = oracle.QSRO(P)
    assert oracle.site_energy(cells, m, occ, 0) == pytest.approx(e0, abs=1e-14)
    assert oracle.site_energy(cells, m, occ, 1) == pytest.approx(e1, abs=1e-14)
    assert oracle.total_energy(cells, m, occ) == pytest.approx(N / 2 * (e0 + e1), abs=1e-11)


def test_single_substitution_closed_form():
    """One species-1 site in pure species 0: the impurity sees only unlike pairs; each of its
    z_m shell-m neighbours has one unlike pair and z_m - 1 like pairs in that shell."""
    P = synth.qsro_params()
    V, W, lam, C = _parts(P)
    cells = (5, 5, 5)
    N = oracle.n_sites(cells)
    pure = np.zeros(N, dtype=np.uint8)
    imp = pure.copy()
    imp[17] = 1
    m = oracle.QSRO(P)
    pure_site = C + W[:, 0].sum() + lam * (W ** 2).sum()
    d_imp = (C + V[0, 1, 0] + V[1, 1, 0] + V[2, 1, 0] + lam * (W ** 2).sum()) - pure_site
    d_nbrs = sum(Z[k] * (V[k - 1, 1, 0] / Z[k] + W[k - 1, 0] * ((Z[k] - 1) / Z[k]) ** 2 - W[k - 1, 0])
                 for k in (1, 2, 3))
    dE = oracle.total_energy(cells, m, imp) - oracle.total_energy(cells, m, pure)
    assert dE == pytest.approx(d_imp + d_nbrs, abs=1e-11)


@pytest.mark.parametrize("cells", [(4, 4, 4), (5, 4, 6)])
def test_qsro_delta_e_equals_total_energy_difference(cells):
    m = oracle.QSRO(synth.qsro_params(n_species=5))
    occ = synth.random_occupancy(cells, 5, None, seed=3)
    rng = np.random.default_rng(2)
    for _ in range(12):
        i = int(rng.integers(occ.size))
        n = oracle.neighbor(cells, i, int(rng.integers(8)))
        after = occ.copy()
        after[i], after[n] = after[n], after[i]
        want = oracle.total_energy(cells, m, after) - oracle.total_energy(cells, m, occ)
        assert oracle.delta_e(cells, m, occ, i, n) == pytest.approx(want, abs=1e-12)


def test_qsro_exact_stationarity_16_sites():
    """pi P_c = pi for the single-trial kernel of both basis sites on the 2x2x2-cell binary
    lattice (12,870 states), with the qSRO energy; periodic images count with multiplicity."""
    cells = (2, 2, 2)
    P = synth.qsro_params(n_species=2)
    P = P * np.float32(20.0)  # a visible energy scale on 16 sites
    m = oracle.QSRO(P)
    from itertools import combinations
    states = []
    for ones in combinations(range(16), 8):
        o = np.zeros(16, dtype=np.uint8)
        o[list(ones)] = 1
        states.append(o)
    E = np.array([oracle.total_energy(cells, m, o) for o in states])
    index = {o.tobytes(): k for k, o in enumerate(states)}
    T = 0.5 * float(np.std(E)) / KB
    beta = 1.0 / (KB * T)
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    for c in (0, 1):
        out = np.zeros_like(pi)
        for k, o in enumerate(states):
            stay = 1.0
            for d in range(8):
                n = oracle.neighbor(cells, c, d)
                if o[c] == o[n]:
                    continue
                a = min(1.0, math.exp(-beta * oracle.delta_e(cells, m, o, c, n)))
                o2 = o.copy()
                o2[c], o2[n] = o[n], o[c]
                out[index[o2.tobytes()]] += pi[k] * a / 8.0
                stay -= a / 8.0
            out[k] += pi[k] * stay
        assert np.max(np.abs(out - pi)) < 1e-12
