"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a library routine (numpy's Philox and
matmul), textbook geometry (BCC coordination 8/6/12 by brute-force distance search),
invariants of the method (dE equals a from-scratch total-energy difference, composition
is conserved, concurrent trials of one colour never touch each other's regions), exact
Boltzmann enumeration on a 16-site lattice, and special cases with closed forms.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth

KB = 8.617333262e-5  # CODATA 2018 Boltzmann constant in eV/K


# ---------------------------------------------------------------------------- helpers
def positions(cells):
    """Doubled-coordinate position of every canonical site, by plain numpy indexing."""
    lx, ly, lz = cells
    s = np.arange(2 * lx * ly * lz)
    b = s % 2
    c = s // 2
    x, y, z = c % lx, (c // lx) % ly, c // (lx * ly)
    return np.stack([2 * x + b, 2 * y + b, 2 * z + b], axis=1)


def brute_neighbor_map(cells, offsets):
    """nbr[s, k] = site at position(s) + offsets[k] (periodic), found by dictionary lookup."""
    P = positions(cells)
    mod = 2 * np.asarray(cells)
    lut = {tuple(p): i for i, p in enumerate(P)}
    out = np.zeros((len(P), len(offsets)), dtype=np.int64)
    for k, d in enumerate(offsets):
        Q = (P + np.asarray(d)) % mod
        out[:, k] = [lut[tuple(q)] for q in Q]
    return out


def small_model(feature, hidden, seed=11, scale=1.0, act0=oracle.ACT_SILU, act1=oracle.ACT_SILU):
    n_in = 12 if feature == oracle.FEAT_COUNTS_S12 else 108
    p = synth.mlp_params(n_in, hidden, seed=seed, scale=scale)
    return oracle.MLP(feature, hidden, p, act0, act1)


# ---------------------------------------------------------------------------- Philox
def test_philox_matches_numpy():
    # numpy.random.Philox is Philox4x64-10; it increments the counter before each block,
    # so its first block for counter c is the block for c + 1.
    rng = np.random.default_rng(123)
    for _ in range(20):
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        ctr[0] = np.uint64(2**64 - 1) if _ == 0 else ctr[0]   # carry into word 1
        bg = np.random.Philox(counter=ctr, key=key)
        want = bg.random_raw(4)
        c = int(ctr[0]) + (int(ctr[1]) << 64) + 1
        nxt = [c & (2**64 - 1), (c >> 64) & (2**64 - 1), int(ctr[2]), int(ctr[3])]
        got = oracle.philox4x64_10(nxt, key)
        assert np.array_equal(got, want)


def test_propose_uses_documented_bits():
    # direction = top 3 bits of r0; u = ((r1 >> 11) + 1) 2^-53
    for site, sweep, rep in [(0, 0, 0), (12345, 7, 3), (2**33 + 5, 199, 95)]:
        r = oracle.philox4x64_10([site, sweep, rep, 0], [0, 0])
        d, u = oracle.propose(0, site, sweep, rep)
        assert d == int(r[0]) >> 61
        assert u == ((int(r[1]) >> 11) + 1) * 2.0**-53
        assert 0.0 < u <= 1.0


# ---------------------------------------------------------------------------- geometry
def test_shells_bruteforce_distance():
    # BCC in doubled coordinates: all-even or all-odd integer points; a = 2 units.
    pts = [p for p in itertools.product(range(-4, 5), repeat=3)
           if len({c % 2 for c in p}) == 1 and p != (0, 0, 0)]
    d2 = np.array([sum(c * c for c in p) for p in pts])
    levels = sorted(set(d2))[:3]
    assert [math.sqrt(v) / 2 for v in levels] == pytest.approx([math.sqrt(3) / 2, 1.0, math.sqrt(2)])
    counts = [int((d2 == v).sum()) for v in levels]
    assert counts == [8, 6, 12]
    off, sh = oracle.shell_table()
    want = []
    for m, v in enumerate(levels):
        want += sorted(p for p, dd in zip(pts, d2) if dd == v)
    assert [tuple(o) for o in off] == want
    assert sh.tolist() == [1] * 8 + [2] * 6 + [3] * 12


@pytest.mark.parametrize("cells", [(5, 6, 7), (4, 4, 4), (2, 2, 2)])
def test_neighbors_match_position_lookup(cells):
    off, _ = oracle.shell_table()
    nb = brute_neighbor_map(cells, off)
    n = oracle.n_sites(cells)
    assert n == 2 * np.prod(cells)
    for s in range(0, n, max(1, n // 97)):
        for k in range(26):
            assert oracle.neighbor(cells, s, k) == nb[s, k]
        assert np.array_equal(oracle.site_pos(cells, s), positions(cells)[s])


def test_features_from_definition():
    cells = (5, 6, 7)
    off, sh = oracle.shell_table()
    nb = brute_neighbor_map(cells, off)
    occ = synth.random_occupancy(cells, n_species=5, seed=3)
    for j in range(0, occ.size, 37):
        x = oracle.features(cells, oracle.FEAT_ONEHOT_S123, occ, j)
        slots = [occ[j]] + [occ[t] for t in nb[j]]
        want = np.zeros(108)
        for m, p in enumerate(slots):
            if p < 4:
                want[4 * m + p] = 1
        assert np.array_equal(x, want)
        xc = oracle.features(cells, oracle.FEAT_COUNTS_S12, occ, j)
        wc = np.zeros(12)
        if occ[j] < 4:
            wc[occ[j]] = 1
        for k in range(14):
            p = occ[nb[j, k]]
            if p < 4:
                wc[(4 if sh[k] == 1 else 8) + p] += 1
        assert np.array_equal(xc, wc)
        # exchanged view: species of i and n trade places
        i, n_ = j, nb[j, 3]
        xs = oracle.features(cells, oracle.FEAT_ONEHOT_S123, occ, nb[j, 20], swap=(i, n_))
        occ2 = occ.copy()
        occ2[i], occ2[n_] = occ[n_], occ[i]
        assert np.array_equal(xs, oracle.features(cells, oracle.FEAT_ONEHOT_S123, occ2, nb[j, 20]))


# ---------------------------------------------------------------------------- model
def silu(z):
    return z / (1.0 + np.exp(-z))


@pytest.mark.parametrize("feature,hidden", [(oracle.FEAT_COUNTS_S12, 64), (oracle.FEAT_ONEHOT_S123, 128)])
def test_mlp_matches_numpy_matmul(feature, hidden):
    m = small_model(feature, hidden)
    F = m.n_in
    p = m.params
    W0 = p[:hidden * F].reshape(hidden, F); o = hidden * F
    b0 = p[o:o + hidden]; o += hidden
    W1 = p[o:o + hidden * hidden].reshape(hidden, hidden); o += hidden * hidden
    b1 = p[o:o + hidden]; o += hidden
    W2 = p[o:o + hidden]; o += hidden
    b2 = p[o]
    rng = np.random.default_rng(0)
    for _ in range(10):
        x = rng.integers(0, 3, size=F).astype(np.float64)
        want = W2 @ silu(W1 @ silu(W0 @ x + b0) + b1) + b2
        assert oracle.mlp(m, x) == pytest.approx(want, rel=1e-13, abs=1e-13)


def test_blob_sizes_match_config():
    assert synth.mlp_n_params(12, 64) == 5057
    assert synth.mlp_n_params(108, 128) == 30593


# ---------------------------------------------------------------------------- Omega
@pytest.mark.parametrize("feature,size", [(oracle.FEAT_COUNTS_S12, 22), (oracle.FEAT_ONEHOT_S123, 40)])
def test_omega_is_set_of_changed_sites(feature, size):
    cells = (6, 6, 6)
    occ = synth.random_occupancy(cells, 4, seed=2)
    n_sites = occ.size
    off, _ = oracle.shell_table()
    for i in [0, 1, 77, 300]:
        for d in range(8):
            n = oracle.neighbor(cells, i, d)
            om = oracle.omega(cells, feature, i, n)
            assert len(om) == size
            # brute force: sites whose feature vector can change, found by giving i and n
            # species that differ in every way and comparing features of every site
            o2 = occ.copy()
            o2[i], o2[n] = 0, 1
            changed = [j for j in range(n_sites)
                       if not np.array_equal(oracle.features(cells, feature, o2, j),
                                             oracle.features(cells, feature, o2, j, swap=(i, n)))]
            assert changed == om.tolist()


@pytest.mark.parametrize("feature,cells", [(oracle.FEAT_COUNTS_S12, (4, 4, 4)),
                                           (oracle.FEAT_ONEHOT_S123, (4, 5, 4)),
                                           (oracle.FEAT_ONEHOT_S123, (2, 2, 2))])
def test_delta_e_equals_total_energy_difference(feature, cells):
    m = small_model(feature, 16)
    occ = synth.random_occupancy(cells, 4, seed=5)
    rng = np.random.default_rng(1)
    e0 = oracle.total_energy(cells, m, occ)
    for _ in range(12):
        i = int(rng.integers(occ.size))
        n = oracle.neighbor(cells, i, int(rng.integers(8)))
        if occ[i] == occ[n]:
            continue
        o2 = occ.copy()
        o2[i], o2[n] = occ[n], occ[i]
        want = oracle.total_energy(cells, m, o2) - e0
        got = oracle.delta_e(cells, m, occ, i, n)
        assert got == pytest.approx(want, abs=1e-12 * abs(e0) + 1e-13)


# ---------------------------------------------------------------------------- schedule
def _read_write_sets(cells, feature, i, n_nb):
    """Write set (i and every possible partner) and read region (Omega of every possible
    partner plus all of their neighbours), by the position lookup of this test file."""
    off, _ = oracle.shell_table()
    nb = _read_write_sets.nb
    writes = {i} | {int(nb[i, d]) for d in range(8)}
    omega = set()
    for d in range(8):
        n = int(nb[i, d])
        omega |= {i, n} | {int(t) for t in nb[i, :n_nb]} | {int(t) for t in nb[n, :n_nb]}
    reads = set(omega)
    for j in omega:
        reads |= {int(t) for t in nb[j, :n_nb]}
    return writes, omega, reads


@pytest.mark.parametrize("cells", [(8, 8, 8), (9, 10, 13), (4, 8, 12)])
def test_schedule_covers_every_site_once_and_is_conflict_free(cells):
    off, _ = oracle.shell_table()
    _read_write_sets.nb = brute_neighbor_map(cells, off)
    col = oracle.colours(cells)
    C = oracle.n_colours(cells)
    e = [max(E // max(1, E // 4) + (1 if E % max(1, E // 4) else 0), 1) for E in cells]
    assert C == 2 * e[0] * e[1] * e[2]
    assert col.min() >= 0 and col.max() < C
    if cells == (8, 8, 8):
        assert C == 128 and np.all(np.bincount(col, minlength=C) == 8)
    for c in range(C):
        members = np.nonzero(col == c)[0]
        sets = [_read_write_sets(cells, 1, int(i), 26) for i in members]
        for a in range(len(members)):
            for b in range(a + 1, len(members)):
                wa, oa, ra = sets[a]
                wb, ob, rb = sets[b]
                assert not (wa & rb) and not (wb & ra) and not (oa & ob)


def test_link_cell_edge_three_would_conflict():
    # Why link cells are at least 4 cells wide: trial sites 3 cells apart can touch.
    cells = (12, 12, 12)
    off, _ = oracle.shell_table()
    _read_write_sets.nb = brute_neighbor_map(cells, off)
    i = 0
    j = 3 * 2  # site index of cell (3,0,0), basis 0
    wa, oa, ra = _read_write_sets(cells, 1, i, 26)
    wb, ob, rb = _read_write_sets(cells, 1, j, 26)
    assert (wa & rb) or (oa & ob)


# ---------------------------------------------------------------------------- rule
def test_metropolis_rule_direction_and_constant():
    rng = np.random.default_rng(9)
    for T in [300.0, 1000.0, 3000.0]:
        for _ in range(2000):
            dE = rng.normal(0, 0.2)
            u = rng.uniform(1e-12, 1.0)
            want = u <= math.exp(-dE / (KB * T))
            if abs(u - math.exp(-dE / (KB * T))) < 1e-9:
                continue
            assert oracle.lib().or_accept(dE, oracle.theta(T, u)) == want
    assert oracle.theta(1000.0, 1.0) == 0.0
    assert math.isinf(oracle.theta(float("inf"), 0.5))


# ---------------------------------------------------------------------------- balance
def _enumerate_binary_16(model):
    cells = (2, 2, 2)
    states = []
    for ones in itertools.combinations(range(16), 8):
        o = np.zeros(16, dtype=np.uint8)
        o[list(ones)] = 1
        states.append(o)
    E = np.array([oracle.total_energy(cells, model, o) for o in states])
    index = {o.tobytes(): k for k, o in enumerate(states)}
    return cells, states, E, index


@pytest.mark.parametrize("feature", [oracle.FEAT_COUNTS_S12, oracle.FEAT_ONEHOT_S123])
def test_exact_stationarity_16_sites(feature):
    """pi P_c = pi exactly for the single-trial kernel of a trial site (both basis sites),
    with pi the Boltzmann distribution over all C(16,8) = 12,870 binary states."""
    model = small_model(feature, 8, seed=21, scale=3.0)
    cells, states, E, index = _enumerate_binary_16(model)
    assert len(states) == 12870
    T = 0.5 * float(np.std(E)) / KB            # beta * std(E) = 2
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
                dE = oracle.delta_e(cells, model, o, c, n)
                a = min(1.0, math.exp(-beta * dE))
                o2 = o.copy()
                o2[c], o2[n] = o[n], o[c]
                out[index[o2.tobytes()]] += pi[k] * a / 8.0
                stay -= a / 8.0
            out[k] += pi[k] * stay
        assert np.max(np.abs(out - pi)) < 1e-12


@pytest.mark.slow
def test_mc_histogram_matches_enumeration_16_sites():
    """The oracle's own sweeps (Philox proposals, theta rule, colour schedule) sample the
    exact Boltzmann energy distribution on the 16-site binary lattice."""
    model = small_model(oracle.FEAT_ONEHOT_S123, 8, seed=21, scale=3.0)
    cells, states, E, _ = _enumerate_binary_16(model)
    T = 0.5 * float(np.std(E)) / KB
    beta = 1.0 / (KB * T)
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    edges = np.quantile(E, np.linspace(0, 1, 9))
    edges[-1] += 1.0
    p_bin = np.array([pi[(E >= edges[b]) & (E < edges[b + 1])].sum() for b in range(8)])
    occ = states[0].copy()
    n_sweeps = 12000
    samples = np.zeros(n_sweeps)
    for t in range(n_sweeps):
        oracle.sweep(cells, model, occ, T, seed=7, replica=0, sweep_index=t)
        samples[t] = oracle.total_energy(cells, model, occ)
    samples = samples[500:]
    hist = np.array([((samples >= edges[b]) & (samples < edges[b + 1])).sum() for b in range(8)])
    frac = hist / hist.sum()
    # blocking estimate of the standard error of each bin fraction
    nb = 50
    blocks = np.array_split(samples, nb)
    bf = np.array([[((blk >= edges[b]) & (blk < edges[b + 1])).mean() for b in range(8)]
                   for blk in blocks])
    se = bf.std(axis=0, ddof=1) / math.sqrt(nb) + 1e-4
    z = (frac - p_bin) / se
    assert np.all(np.abs(z) < 5.0), (frac, p_bin, z)


# ---------------------------------------------------------------------------- invariants
def _c1_like(hidden=16, cells=(8, 8, 8)):
    m = small_model(oracle.FEAT_COUNTS_S12, hidden, seed=1)
    occ = synth.random_occupancy(cells, 4, seed=0)
    return cells, m, occ


def test_composition_conserved_and_running_total_equals_scratch():
    cells, m, occ = _c1_like()
    e0 = oracle.total_energy(cells, m, occ)
    st = oracle.Stats()
    st.e_run = e0
    counts0 = np.bincount(occ, minlength=4)
    for t in range(4):
        oracle.sweep(cells, m, occ, 1000.0, 0, 0, t, stats=st)
        assert np.array_equal(np.bincount(occ, minlength=4), counts0)
    assert st.attempts == 4 * occ.size
    assert st.accepts > 0
    assert st.e_run == pytest.approx(oracle.total_energy(cells, m, occ), abs=1e-9 * abs(e0))


def test_trial_order_inside_a_colour_does_not_matter():
    cells, m, occ = _c1_like(cells=(8, 12, 8))
    ref = occ.copy()
    _, tr_ref = oracle.sweep(cells, m, ref, 800.0, 3, 0, 0, trace=True,
                             order=oracle.ORDER_SNAPSHOT, nthreads=4)
    perm = np.random.default_rng(0).permutation(occ.size)
    for order, given in [(oracle.ORDER_FORWARD, None), (oracle.ORDER_REVERSE, None),
                         (oracle.ORDER_GIVEN, perm)]:
        o = occ.copy()
        _, tr = oracle.sweep(cells, m, o, 800.0, 3, 0, 0, trace=True, order=order,
                             given_order=given)
        assert np.array_equal(o, ref)
        assert np.array_equal(tr, tr_ref)


def test_double_lattice_reduction_equals_per_trial_delta_e():
    """Algorithm 1 literally: sigma1 = sigma0 with every trial of one colour swapped,
    local energies of all sites on both lattices, reduce each over its Omega."""
    cells = (8, 8, 8)
    m = small_model(oracle.FEAT_ONEHOT_S123, 16, seed=4)
    occ = synth.random_occupancy(cells, 4, seed=8)
    col = oracle.colours(cells)
    e0_all = oracle.all_site_energies(cells, m, occ)
    for c in [0, 1, 77]:
        recs = [oracle.trial(cells, m, occ, 1000.0, 0, 0, 0, int(s)) for s in np.nonzero(col == c)[0]]
        sigma1 = occ.copy()
        for r in recs:
            sigma1[r["site"]], sigma1[r["partner"]] = occ[r["partner"]], occ[r["site"]]
        e1_all = oracle.all_site_energies(cells, m, sigma1)
        for r in recs:
            om = oracle.omega(cells, oracle.FEAT_ONEHOT_S123, r["site"], r["partner"])
            dE = float(np.sum(e1_all[om] - e0_all[om]))
            assert dE == pytest.approx(r["dE"], abs=1e-12)


def test_infinite_temperature_accepts_every_different_species_trial():
    cells, m, occ = _c1_like()
    st, tr = oracle.sweep(cells, m, occ, float("inf"), 0, 0, 0, trace=True)
    assert st.accepts == st.diff_species
    assert np.all(tr["accept"] == 1 - tr["same"])


def test_zero_temperature_never_raises_energy():
    cells, m, occ = _c1_like()
    _, tr = oracle.sweep(cells, m, occ, 0.0, 0, 0, 0, trace=True)
    assert np.all(tr["dE"][tr["accept"] == 1] <= 0.0)


def test_zero_weights_give_zero_delta_e():
    cells = (6, 6, 6)
    m = oracle.MLP(oracle.FEAT_ONEHOT_S123, 16, np.zeros(synth.mlp_n_params(108, 16)))
    occ = synth.random_occupancy(cells, 4, seed=1)
    _, tr = oracle.sweep(cells, m, occ, 500.0, 0, 0, 0, trace=True)
    assert np.all(tr["dE"] == 0.0)
    assert np.all(tr["accept"] == 1 - tr["same"])


@pytest.mark.parametrize("feature", [oracle.FEAT_COUNTS_S12, oracle.FEAT_ONEHOT_S123])
def test_linear_model_is_translation_invariant_point_model(feature):
    """With identity activations the energy is linear in the features, and every feature
    slot is a translate of the lattice, so the total energy only depends on composition:
    every swap has dE = 0.  A wrong neighbour map (not a bijection) breaks this."""
    cells = (6, 7, 8)
    m = small_model(feature, 16, seed=3, act0=oracle.ACT_IDENTITY, act1=oracle.ACT_IDENTITY)
    occ = synth.random_occupancy(cells, 4, seed=2)
    rng = np.random.default_rng(0)
    for _ in range(20):
        i = int(rng.integers(occ.size))
        n = oracle.neighbor(cells, i, int(rng.integers(8)))
        assert abs(oracle.delta_e(cells, m, occ, i, n)) < 1e-12


def test_quadratic_model_matches_pair_expansion():
    """Square activation after layer 0, identity after layer 1 with W1 = I and b1 = 0:
    E_j = sum_h w2_h (b0_h + sum_m W0[h, slot m species])^2 + b2, a sum of pair terms over
    the 27-site cluster of j.  The total energy computed as that pair sum over every
    cluster must equal the oracle's total energy."""
    cells = (4, 4, 5)
    H = 6
    F = 108
    rng = np.random.default_rng(2)
    W0 = rng.normal(size=(H, F)); b0 = rng.normal(size=H)
    W1 = np.eye(H); b1 = np.zeros(H); W2 = rng.normal(size=H); b2 = rng.normal(size=1)
    blob = np.concatenate([W0.ravel(), b0, W1.ravel(), b1, W2, b2])
    m = oracle.MLP(oracle.FEAT_ONEHOT_S123, H, blob, oracle.ACT_SQUARE, oracle.ACT_IDENTITY)
    occ = synth.random_occupancy(cells, 4, seed=4)
    off, _ = oracle.shell_table()
    nb = brute_neighbor_map(cells, off)
    # column of W0 selected by (slot m, species p)
    total = 0.0
    for j in range(occ.size):
        slots = [occ[j]] + [occ[t] for t in nb[j]]
        cols = [4 * m_ + p for m_, p in enumerate(slots)]
        # (b0 + sum_m W0[:, c_m])^2 = b0^2 + 2 b0 sum_m W0c_m + sum_{m,m'} W0c_m W0c_m'
        ej = W2 @ (b0 * b0) + b2[0]
        for a in cols:
            ej += 2.0 * W2 @ (b0 * W0[:, a])
            for b in cols:
                ej += W2 @ (W0[:, a] * W0[:, b])
        total += ej
    assert total == pytest.approx(oracle.total_energy(cells, m, occ), rel=1e-12)


# ---------------------------------------------------------------------------- observables
def test_warren_cowley_of_b2_order():
    """Perfect B2 (CsCl) order: species 0 on basis 0, species 1 on basis 1.  Shell 1 joins
    the two sublattices, shells 2 and 3 stay inside one: alpha1^{00} = 1, alpha1^{01} = -1,
    alpha2^{00} = -1, alpha2^{01} = 1 (c = 1/2)."""
    cells = (4, 4, 4)
    occ = (np.arange(128) % 2).astype(np.uint8)
    a = oracle.warren_cowley(cells, occ, 2)
    assert a[0].tolist() == [[1.0, -1.0], [-1.0, 1.0]]
    assert a[1].tolist() == [[-1.0, 1.0], [1.0, -1.0]]
    assert a[2].tolist() == [[-1.0, 1.0], [1.0, -1.0]]


def test_equiatomic_counts_largest_remainder():
    c = synth.species_counts(33554432, np.full(5, 0.2))
    assert c.tolist() == [6710887, 6710887, 6710886, 6710886, 6710886]
    occ = synth.random_occupancy((8, 8, 8), 4)
    assert np.bincount(occ).tolist() == [256] * 4


def test_batched_proposals_follow_the_philox_definition():
    """Batched proposals against numpy's Philox4x64-10 (a library routine) and a brute-force
    neighbour lookup: slot = r0 >> 61, theta = -kB T ln(((r1 >> 11) + 1) 2^-53)."""
    cells = (5, 6, 7)
    sites = np.arange(0, oracle.n_sites(cells), 7)
    T, seed, sweep_index, replica = 900.0, 11, 3, 2
    d, p, th = oracle.proposals(cells, seed, replica, sweep_index, T, sites)
    off, _ = oracle.shell_table()
    nbr = brute_neighbor_map(cells, off[:8])
    for a, s in enumerate(sites[:200]):
        # numpy's block for counter c is the block of c + 1 (it increments before drawing)
        ctr = np.array([int(s), sweep_index, replica, 0], dtype=np.uint64)
        bg = np.random.Philox(counter=_counter_minus_one(ctr), key=np.array([seed, 0], dtype=np.uint64))
        r = bg.random_raw(4)
        assert d[a] == int(r[0]) >> 61
        u = ((int(r[1]) >> 11) + 1) * 2.0 ** -53
        assert th[a] == pytest.approx(-KB * T * math.log(u), rel=1e-15, abs=1e-300)
        assert p[a] == nbr[s, d[a]]


def _counter_minus_one(ctr):
    c = [int(v) for v in ctr]
    for k in range(4):
        if c[k] > 0:
            c[k] -= 1
            break
        c[k] = 2 ** 64 - 1
    return np.array(c, dtype=np.uint64)


def test_forced_decisions():
    """An imposed decision replaces the Metropolis one: imposing every trial's own decision
    changes nothing; imposing acceptance everywhere is the T = +inf sweep; imposing rejection
    everywhere leaves the lattice as it was; imposing one flipped decision changes exactly
    that pair of its colour and nothing before it."""
    cells, m, occ0 = _c1_like()
    ref = occ0.copy()
    _, tr = oracle.sweep(cells, m, ref, 800.0, 0, 0, 0, trace=True)
    o = occ0.copy()
    own = np.where(tr["same"] == 1, -1, tr["accept"]).astype(np.int8)
    _, tr2 = oracle.sweep(cells, m, o, 800.0, 0, 0, 0, trace=True, force=own)
    assert np.array_equal(o, ref) and np.array_equal(tr2["accept"], tr["accept"])
    o, inf = occ0.copy(), occ0.copy()
    oracle.sweep(cells, m, o, 800.0, 0, 0, 0, force=np.ones(o.size, dtype=np.int8))
    oracle.sweep(cells, m, inf, float("inf"), 0, 0, 0)
    assert np.array_equal(o, inf)
    o = occ0.copy()
    oracle.sweep(cells, m, o, 800.0, 0, 0, 0, force=np.zeros(o.size, dtype=np.int8))
    assert np.array_equal(o, occ0)
    # flip the first different-species trial of the last colour: only that pair changes
    C = oracle.n_colours(cells)
    last = [s for s in np.nonzero(tr["colour"] == C - 1)[0] if tr["same"][s] == 0][0]
    f = np.full(o.size, -1, dtype=np.int8)
    f[last] = 1 - tr["accept"][last]
    o = occ0.copy()
    _, tr3 = oracle.sweep(cells, m, o, 800.0, 0, 0, 0, trace=True, force=f)
    changed = np.nonzero(o != ref)[0]
    assert set(changed) == {last, tr["partner"][last]}
    assert tr3["accept"][last] == 1 - tr["accept"][last]
    assert tr3["dE"][last] == tr["dE"][last]
