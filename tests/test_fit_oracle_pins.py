"""Pins of the differentiation-pattern oracle (cluster-expansion labels, fit loss and its
gradient) against facts that do not come from the oracle itself: brute-force enumeration,
closed forms on an ordered structure, central finite differences, and PyTorch's CPU autograd
(a library routine) on an FP64 copy of the model."""
import numpy as np
import pytest

import oracle
import synth


def ce_model(n_species=4, **kw):
    p = synth.ce_params(n_species=n_species, **kw)
    tri = oracle.ce_triangles()
    return oracle.CEModel(p["n_species"], p["pair"], tri[p["triangle"]], p["species"], p["J"]), p


def test_triangle_shapes_brute_force():
    """Canonical triangle shapes with all edges within shell 3, recounted by brute force over
    site triples of a periodic 6^3 lattice around one site."""
    tri = oracle.ce_triangles()
    assert len(tri) == synth.N_CE_TRIANGLES
    off, _ = oracle.shell_table()
    near = [tuple(o) for o in off]
    shapes = set()
    d2ok = {3, 4, 8}
    for a in near:
        for b in near:
            if a == b:
                continue
            d = tuple(x - y for x, y in zip(a, b))
            if sum(v * v for v in d) not in d2ok:
                continue
            pts = sorted([(0, 0, 0), a, b])
            o = pts[0]
            shapes.add(tuple(x - y for p in pts[1:] for x, y in zip(p, o)))
    assert sorted(shapes) == [tuple(t) for t in tri]
    # every shape: three pairwise squared distances in {3, 4, 8}
    for t in tri:
        a, b = t[:3], t[3:]
        for v in (a, b, a - b):
            assert int((v * v).sum()) in d2ok


@pytest.mark.parametrize("cells", [(4, 4, 4), (5, 4, 6)])
def test_ce_local_sum_equals_brute_force(cells):
    ce, _ = ce_model()
    for seed in range(3):
        occ = synth.random_occupancy(cells, 4, [0.4, 0.3, 0.2, 0.1], seed=seed)
        e_loc = oracle.ce_total(cells, ce, occ)
        e_bf = oracle.ce_total(cells, ce, occ, brute=True)
        assert e_loc == pytest.approx(e_bf, abs=1e-12 * max(1.0, abs(e_bf)))


def test_ce_b2_closed_form():
    """Perfect B2 order (species 0 on corners, 1 on body centres): shell-1 pairs are all
    (0,1), 4N of them; shells 2 and 3 pair like with like, 3N and 6N pairs split evenly; a
    triangle item matches at the N/2 origins of each sublattice whose parity pattern fits."""
    ce, p = ce_model()
    cells = (4, 4, 4)
    N = oracle.n_sites(cells)
    occ = (np.arange(N) % 2).astype(np.uint8)
    V = p["pair"]
    want = 4 * N * V[0, 0, 1] + 1.5 * N * (V[1, 0, 0] + V[1, 1, 1]) + 3 * N * (V[2, 0, 0] + V[2, 1, 1])
    tri = oracle.ce_triangles()[p["triangle"]]
    for t, sp, J in zip(tri, p["species"], p["J"]):
        for s0 in (0, 1):
            s1 = s0 ^ (int(t[0]) & 1)
            s2 = s0 ^ (int(t[3]) & 1)
            if (s0, s1, s2) == tuple(int(v) for v in sp):
                want += J * N / 2
    assert oracle.ce_total(cells, ce, occ) == pytest.approx(want, abs=1e-12)
    assert oracle.ce_total(cells, ce, occ, brute=True) == pytest.approx(want, abs=1e-12)


def test_ce_swap_changes_only_nearby_sites():
    """A swap changes the local CE energies only of sites within shell 3 of the pair
    (locality that makes the CE learnable by the 27-site MLP), and the total change equals
    the sum of the local changes."""
    ce, _ = ce_model()
    cells = (5, 5, 5)
    occ = synth.random_occupancy(cells, 4, None, seed=7)
    N = occ.size
    e0 = np.array([oracle.ce_site_energy(cells, ce, occ, s) for s in range(N)])
    i = 17
    n = oracle.neighbor(cells, i, 3)
    occ1 = occ.copy()
    occ1[i], occ1[n] = occ1[n], occ1[i]
    e1 = np.array([oracle.ce_site_energy(cells, ce, occ1, s) for s in range(N)])
    changed = set(np.nonzero(np.abs(e1 - e0) > 0)[0].tolist())
    near = {i, n} | {oracle.neighbor(cells, i, k) for k in range(26)} | {oracle.neighbor(cells, n, k) for k in range(26)}
    assert changed <= near
    dE = oracle.ce_total(cells, ce, occ1, brute=True) - oracle.ce_total(cells, ce, occ, brute=True)
    assert (e1 - e0).sum() == pytest.approx(dE, abs=1e-12)


def _fit_case(cells=(4, 4, 4), batch=2, scale=1.0):
    params = synth.mlp_params(108, 128, seed=11, scale=scale)
    model = oracle.MLP(1, 128, params)
    snaps = synth.snapshots(batch, cells[0], seed=21)
    ce, _ = ce_model()
    labels = np.array([oracle.ce_total(cells, ce, s) for s in snaps])
    return model, snaps, labels


def test_fit_gradient_matches_central_differences():
    """1,000 parameters drawn with the FD seed (every block of the blob represented)."""
    cells = (4, 4, 4)
    model, snaps, labels = _fit_case(cells)
    loss, S, g = oracle.fit_loss_grad(cells, model, snaps, labels)
    P = model.params.size
    rng = np.random.default_rng(synth.SEED_FD)
    idx = np.sort(rng.choice(P, size=1000, replace=False))
    # make sure the biases and the output layer are among them
    idx = np.unique(np.concatenate([idx, [128 * 108, 128 * 108 + 5, P - 129, P - 2, P - 1]]))
    fd = oracle.fit_fd(cells, model, snaps, labels, idx, h=1e-6)
    err = np.abs(fd - g[idx])
    assert np.all(err <= 1e-6 * np.abs(g[idx]) + 2e-9), (err.max(), idx[np.argmax(err)])
    assert loss > 0 and np.linalg.norm(g) > 0


def test_fit_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    cells = (4, 4, 4)
    model, snaps, labels = _fit_case(cells, batch=3)
    loss, S, g = oracle.fit_loss_grad(cells, model, snaps, labels)
    N = snaps.shape[1]
    X = np.stack([np.stack([oracle.features(cells, 1, s, j) for j in range(N)]) for s in snaps])
    p = torch.tensor(model.params, dtype=torch.float64, requires_grad=True)
    H, F = 128, 108
    W0 = p[:H * F].view(H, F)
    b0 = p[H * F:H * F + H]
    o = H * F + H
    W1 = p[o:o + H * H].view(H, H)
    b1 = p[o + H * H:o + H * H + H]
    o += H * H + H
    W2 = p[o:o + H]
    b2 = p[o + H]
    x = torch.tensor(X, dtype=torch.float64)
    h1 = torch.nn.functional.silu(x @ W0.T + b0)
    h2 = torch.nn.functional.silu(h1 @ W1.T + b1)
    E = h2 @ W2 + b2
    St = E.sum(dim=1)
    lt = (((St - torch.tensor(labels)) / N) ** 2).mean()
    lt.backward()
    assert St.detach().numpy() == pytest.approx(S, rel=1e-12)
    assert float(lt.detach()) == pytest.approx(loss, rel=1e-12)
    gt = p.grad.numpy()
    assert np.allclose(g, gt, rtol=1e-9, atol=1e-15 * np.abs(gt).max())


def test_energy_grad_is_linear_in_upstream():
    cells = (4, 4, 4)
    model, snaps, _ = _fit_case(cells, batch=2)
    ga = oracle.energy_grad(cells, model, snaps, [1.0, 0.0])
    gb = oracle.energy_grad(cells, model, snaps, [0.0, 1.0])
    gc = oracle.energy_grad(cells, model, snaps, [2.0, -3.0])
    assert np.allclose(gc, 2 * ga - 3 * gb, rtol=1e-12, atol=1e-14)
    # the output bias enters each site once: dS/db2 = N
    assert ga[-1] == pytest.approx(snaps.shape[1])


@pytest.mark.parametrize("S", [4, 5])
def test_ce_pair_qsro_carries_the_ce_pair_part(S):
    """The qSRO blob built from a CE's pair terms (the driving model of the snapshot chains):
    the oracle's qSRO energy differs from the oracle's CE pair energy by the composition term
    sum_i sum_m (z_m / 2) pair_m(s_i, s_i) (closed form), so any species exchange changes both
    by the same amount."""
    from paper_2604_08250_amd.fit import BCC_SHELL_SIZES, ce_pair_qsro
    p = synth.ce_params(n_species=S)
    pair = p["pair"]
    ce = oracle.CEModel(S, pair, np.zeros((0, 6)), np.zeros((0, 3)), np.zeros(0))
    q = oracle.QSRO(ce_pair_qsro(pair))
    cells = (4, 5, 6)
    occ = synth.random_occupancy(cells, S, seed=71)
    rng = np.random.default_rng(72)

    def const(o):
        return sum(BCC_SHELL_SIZES[m] / 2.0 * pair[m][o, o].sum() for m in range(3))

    # blob entries are FP32: agreement to the rounding of about 40 pair terms of ~0.1 eV
    tol = 2e-6
    e_ce, e_q = oracle.ce_total(cells, ce, occ), oracle.total_energy(cells, q, occ)
    assert e_ce - e_q == pytest.approx(const(occ), abs=tol * occ.size)
    for _ in range(40):
        i, n = rng.choice(occ.size, size=2, replace=False)
        nxt = occ.copy()
        nxt[i], nxt[n] = occ[n], occ[i]
        d_ce = oracle.ce_total(cells, ce, nxt) - e_ce
        d_q = oracle.total_energy(cells, q, nxt) - e_q
        assert d_q == pytest.approx(d_ce, abs=tol)


def test_ce_pair_qsro_additive_pairs_are_flat():
    """A CE whose pair terms are additive, pair_m(p, q) = (a_m(p) + a_m(q)) / 2, has the energy
    sum_m (z_m / 2) sum_i a_m(s_i), fixed by the composition: its qSRO blob is zero, and no
    exchange changes the CE energy (oracle)."""
    from paper_2604_08250_amd.fit import BCC_SHELL_SIZES, ce_pair_qsro
    S = 4
    a = np.random.default_rng(73).normal(0.0, 0.03, size=(3, S))
    pair = 0.5 * (a[:, :, None] + a[:, None, :])
    assert not np.any(ce_pair_qsro(pair))
    ce = oracle.CEModel(S, pair, np.zeros((0, 6)), np.zeros((0, 3)), np.zeros(0))
    cells = (4, 4, 5)
    occ = synth.random_occupancy(cells, S, seed=74)
    e0 = oracle.ce_total(cells, ce, occ)
    assert e0 == pytest.approx(sum(BCC_SHELL_SIZES[m] / 2.0 * a[m][occ].sum() for m in range(3)), abs=1e-10)
    rng = np.random.default_rng(75)
    for _ in range(10):
        i, n = rng.choice(occ.size, size=2, replace=False)
        occ[i], occ[n] = occ[n], occ[i]
        assert oracle.ce_total(cells, ce, occ) == pytest.approx(e0, abs=1e-10)
