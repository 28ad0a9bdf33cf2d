"""Pins of the FCC oracle (geometry, MLPNet of Eqs. (4)-(6), qSRO of Eq. 2 over FCC shells,
colouring, sweeps) against what does not come from the oracle itself: positions and shells
from a brute-force minimum-image distance search, MLPNet against torch's Linear/ReLU layers,
closed forms worked out by hand on the L1_2 structure, independence of same-colour trials by
brute force, and exact Boltzmann stationarity on a 16-site lattice."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import ORDER_FORWARD, ORDER_REVERSE, ORDER_SNAPSHOT, KB_EV_PER_K
from oracle import fcc

BASIS = np.array([[0, 0, 0], [0, 1, 1], [1, 0, 1], [1, 1, 0]])


def _positions(cells):
    lx, ly, lz = cells
    out = []
    for z, y, x, b in itertools.product(range(lz), range(ly), range(lx), range(4)):
        out.append(2 * np.array([x, y, z]) + BASIS[b])
    return np.array(out)


def _min_image(d, cells):
    per = 2 * np.asarray(cells)
    return (d + per // 2) % per - per // 2


def test_fcc_positions_and_index():
    cells = (4, 5, 6)
    P = _positions(cells)
    assert fcc.n_sites(cells) == len(P) == 480
    for s in range(len(P)):
        assert np.array_equal(fcc.site_pos(cells, s), P[s])
        assert fcc.site_at(cells, P[s]) == s
    assert np.all(P.sum(axis=1) % 2 == 0)
    assert len({tuple(p) for p in P}) == len(P)
    assert fcc.site_at(cells, (1, 0, 0)) == -1


def test_fcc_shells_by_distance():
    """Slots 0-11, 12-17 and 18-41 are the sites at squared doubled distance 2, 4 and 6
    (a/sqrt2, a, a*sqrt(3/2)): 12, 6 and 24 of them; each shell in lexicographic order."""
    cells = (6, 6, 6)
    P = _positions(cells)
    off, sh = fcc.shell_table()
    assert sh.tolist() == [1] * 12 + [2] * 6 + [3] * 24
    for shell, lo, hi in ((1, 0, 12), (2, 12, 18), (3, 18, 42)):
        assert off[lo:hi].tolist() == sorted(off[lo:hi].tolist())
    rng = np.random.default_rng(0)
    for s in rng.integers(len(P), size=12):
        d = _min_image(P - P[s], cells)
        d2 = (d ** 2).sum(axis=1)
        for want_d2, lo, hi in ((2, 0, 12), (4, 12, 18), (6, 18, 42)):
            brute = set(np.nonzero(d2 == want_d2)[0].tolist())
            got = {fcc.neighbor(cells, int(s), k) for k in range(lo, hi)}
            assert got == brute and len(brute) == hi - lo
        # and the slot order is the lexicographic order of the offsets
        for k in range(42):
            n = fcc.neighbor(cells, int(s), k)
            assert np.array_equal(_min_image(P[n] - P[s], cells), off[k])


def test_fcc_features_by_brute_force():
    cells = (6, 6, 6)
    P = _positions(cells)
    occ = synth.random_occupancy(cells, 5, synth.HEA_COMPOSITION, seed=2, basis=4)
    for j in (0, 7, 301, 863):
        d = _min_image(P - P[j], cells)
        d2 = (d ** 2).sum(axis=1)
        nbrs = [n for n in range(len(P)) if d2[n] in (2, 4)]
        nbrs.sort(key=lambda n: (d2[n], tuple(d[n])))
        x = np.zeros(76)
        for slot, s in enumerate([j] + nbrs):
            if occ[s] < 4:
                x[4 * slot + occ[s]] = 1.0
        assert np.array_equal(fcc.features(cells, occ, j), x)


def test_mlpnet_equals_torch_layers():
    torch = pytest.importorskip("torch")
    H = 96
    blob = synth.mlpnet_params(H, seed=3).astype(np.float64)
    model = fcc.MLPNet(H, blob)
    sizes = synth.mlpnet_param_sizes(H)
    parts, at = {}, 0
    for name, shape, _ in sizes:
        n = int(np.prod(shape))
        parts[name] = torch.tensor(blob[at:at + n].reshape(shape))
        at += n
    net = torch.nn.Sequential(torch.nn.Linear(76, H), torch.nn.ReLU(), torch.nn.Linear(H, H), torch.nn.ReLU(),
                              torch.nn.Linear(H, H), torch.nn.ReLU(), torch.nn.Linear(H, 1)).double()
    with torch.no_grad():
        for k, li in enumerate((0, 2, 4, 6)):
            net[li].weight.copy_(parts[f"W{k}"])
            net[li].bias.copy_(parts[f"b{k}"])
    rng = np.random.default_rng(4)
    xs = [rng.normal(size=76), (rng.random(76) < 0.25).astype(float)]
    occ = synth.random_occupancy((4, 4, 4), 4, None, seed=1, basis=4)
    xs += [fcc.features((4, 4, 4), occ, j) for j in (0, 100, 255)]
    for x in xs:
        with torch.no_grad():
            want = float(net(torch.tensor(x)[None])[0, 0])
        assert fcc.mlpnet(model, x) == pytest.approx(want, rel=1e-13, abs=1e-13)


def _qsro_parts(P):
    P = np.asarray(P, dtype=np.float64)
    return P[:75].reshape(3, 5, 5), P[75:90].reshape(3, 5), P[90], P[91]


def _l12(cells):
    """L1_2 (A3B): species 1 on the cube corners (basis 0), species 0 on the face centres."""
    n = fcc.n_sites(cells)
    return (np.arange(n) % 4 == 0).astype(np.uint8)


def test_qsro_fcc_closed_forms():
    """Worked by hand.  Pure element: every pair like.  L1_2: a corner site has 12 face-centre
    nearest neighbours, 6 corner second neighbours and 24 face-centre third neighbours; a
    face-centre site has 4 + 8 (corner + face) first, 6 face second and 8 + 16 third."""
    P = synth.qsro_params(n_species=2)
    V, W, lam, C = _qsro_parts(P)
    m = fcc.QSRO(P)
    reg = lam * (W ** 2).sum()
    cells = (4, 4, 4)
    pure = np.zeros(fcc.n_sites(cells), dtype=np.uint8)
    assert fcc.site_energy(cells, m, pure, 5) == pytest.approx(C + W[:, 0].sum() + reg, abs=1e-14)
    occ = _l12(cells)
    e_corner = C + V[0, 1, 0] + W[1, 1] + V[2, 1, 0] + reg
    e_face = C + V[0, 1, 0] / 3 + W[0, 0] * (2 / 3) ** 2 + W[1, 0] + V[2, 1, 0] / 3 + W[2, 0] * (2 / 3) ** 2 + reg
    assert fcc.site_energy(cells, m, occ, 0) == pytest.approx(e_corner, abs=1e-14)
    for b in (1, 2, 3):
        assert fcc.site_energy(cells, m, occ, 4 * 9 + b) == pytest.approx(e_face, abs=1e-14)
    N = occ.size
    assert fcc.total_energy(cells, m, occ) == pytest.approx(N / 4 * (e_corner + 3 * e_face), abs=1e-11)


def test_warren_cowley_fcc_l12():
    """L1_2: P(B in shell 1 | A) = 1/3, c_B = 1/4 -> alpha_1^{AB} = -1/3; shell 2 of A is all A
    -> alpha_2^{AB} = 1; shell 3 of A holds 8 of 24 B -> alpha_3^{AB} = -1/3;
    P(A in shell 1 | B) = 1, c_A = 3/4 -> alpha_1^{BA} = -1/3."""
    a = fcc.warren_cowley((4, 4, 4), _l12((4, 4, 4)), 2)
    assert a[0, 0, 1] == pytest.approx(-1 / 3)
    assert a[1, 0, 1] == pytest.approx(1.0)
    assert a[2, 0, 1] == pytest.approx(-1 / 3)
    assert a[0, 1, 0] == pytest.approx(-1 / 3)
    assert a[1, 1, 1] == pytest.approx(-3.0)  # B's second shell is all B: 1 - 1 / (1/4)


@pytest.mark.parametrize("kind", ["mlpnet", "qsro"])
def test_fcc_delta_e_equals_total_energy_difference(kind):
    cells = (4, 5, 4)
    if kind == "mlpnet":
        m = fcc.MLPNet(96, synth.mlpnet_params(96))
    else:
        m = fcc.QSRO(synth.qsro_params(n_species=5))
    occ = synth.random_occupancy(cells, 5, synth.HEA_COMPOSITION, seed=9, basis=4)
    rng = np.random.default_rng(2)
    base = fcc.total_energy(cells, m, occ)
    for _ in range(8):
        i = int(rng.integers(occ.size))
        n = fcc.neighbor(cells, i, int(rng.integers(12)))
        after = occ.copy()
        after[i], after[n] = after[n], after[i]
        want = fcc.total_energy(cells, m, after) - base
        assert fcc.delta_e(cells, m, occ, i, n) == pytest.approx(want, abs=1e-11)


def test_fcc_zone_sizes():
    cells = (8, 8, 8)
    for d in range(12):
        n = fcc.neighbor(cells, 100, d)
        assert len(fcc.omega(cells, fcc.MLPNET_S12, 100, n)) == 28
        assert len(fcc.omega(cells, fcc.QSRO_S123, 100, n)) == 60


def test_fcc_colours_independent_trials():
    """256 colours on 4x4x4 link cells; on a mixed 4/5 lattice the colour classes are the
    link-cell offsets x basis, and no trial of a colour (any of its 12 partners) writes a site
    that another trial of the colour reads (its zone and the zone's neighbours)."""
    assert fcc.n_colours((4, 4, 4)) == 256
    assert fcc.n_colours((8, 12, 4)) == 256
    cells = (8, 9, 13)
    assert fcc.n_colours(cells) == 4 * 4 * 5 * 5
    col = fcc.colours(cells)
    N = fcc.n_sites(cells)
    assert sorted(set(col.tolist())) == list(range(fcc.n_colours(cells)))
    nb = np.array([[fcc.neighbor(cells, s, k) for k in range(42)] for s in range(N)])
    for c in (0, 77, 399):
        sites = np.nonzero(col == c)[0]
        reads, writes = {}, {}
        for i in sites:
            r, w = set(), {int(i)}
            for d in range(12):
                n = int(nb[i, d])
                w.add(n)
                for o in fcc.omega(cells, fcc.QSRO_S123, int(i), n):
                    r.add(int(o))
                    r.update(nb[o].tolist())
            reads[int(i)], writes[int(i)] = r, w
        for i, j in itertools.combinations(sites.tolist(), 2):
            assert not (writes[i] & reads[j]) and not (writes[j] & reads[i]), (c, i, j)


@pytest.mark.parametrize("kind", ["mlpnet", "qsro"])
def test_fcc_sweep_order_independence(kind):
    cells = (8, 8, 8)
    m = fcc.MLPNet(24, synth.mlpnet_params(24, seed=5)) if kind == "mlpnet" else fcc.QSRO(synth.qsro_params(5))
    occ0 = synth.random_occupancy(cells, 5, synth.HEA_COMPOSITION, seed=4, basis=4)
    outs = []
    for order in (ORDER_SNAPSHOT, ORDER_FORWARD, ORDER_REVERSE):
        occ = occ0.copy()
        st, tr = fcc.sweep(cells, m, occ, 700.0, 11, 0, 0, trace=True, order=order, nthreads=8)
        outs.append((occ, tr, st.accepts))
    for occ, tr, acc in outs[1:]:
        assert np.array_equal(occ, outs[0][0])
        assert np.array_equal(tr["accept"], outs[0][1]["accept"])
        assert acc == outs[0][2] > 0


def test_fcc_proposal_directions_uniform():
    d = np.array([fcc.propose(0, s, 0, 0)[0] for s in range(24000)])
    assert d.min() == 0 and d.max() == 11
    counts = np.bincount(d, minlength=12)
    chi2 = ((counts - 2000.0) ** 2 / 2000.0).sum()
    assert chi2 < 35.0  # 11 degrees of freedom, p ~ 2e-4


@pytest.mark.parametrize("kind", ["mlpnet", "qsro"])
def test_fcc_exact_stationarity_16_sites(kind):
    """pi P_c = pi for the single-trial kernel (12 partners, Metropolis) of sites of the
    2x2x1-cell binary lattice (12,870 states); periodic images count with multiplicity."""
    cells = (2, 2, 1)
    if kind == "mlpnet":
        m = fcc.MLPNet(8, synth.mlpnet_params(8, seed=6) * np.float32(4.0))
    else:
        m = fcc.QSRO(synth.qsro_params(n_species=2) * np.float32(20.0))
    states = []
    for ones in itertools.combinations(range(16), 8):
        o = np.zeros(16, dtype=np.uint8)
        o[list(ones)] = 1
        states.append(o)
    E = np.array([fcc.total_energy(cells, m, o) for o in states])
    index = {o.tobytes(): k for k, o in enumerate(states)}
    T = 0.5 * float(np.std(E)) / KB_EV_PER_K
    beta = 1.0 / (KB_EV_PER_K * T)
    pi = np.exp(-beta * (E - E.min()))
    pi /= pi.sum()
    for c in ((0, 3) if kind == "qsro" else (1, 2)):  # the four basis sites between the two models
        out = np.zeros_like(pi)
        for k, o in enumerate(states):
            stay = 1.0
            for d in range(12):
                n = fcc.neighbor(cells, c, d)
                if o[c] == o[n]:
                    continue
                a = min(1.0, math.exp(-beta * fcc.delta_e(cells, m, o, c, n)))
                o2 = o.copy()
                o2[c], o2[n] = o[n], o[c]
                out[index[o2.tobytes()]] += pi[k] * a / 12.0
                stay -= a / 12.0
            out[k] += pi[k] * stay
        assert np.max(np.abs(out - pi)) < 1e-12
