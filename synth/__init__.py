"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws inputs: species placements, compositions, model parameters,
replica sets and temperatures.  It holds none of the method's arithmetic (no
geometry, no energies, no random-number stream of the Monte Carlo itself), so the
CPU oracle and the HIP path can both take their inputs from here without sharing
any computation.

Workloads (the paper's FCC FeCoNiAlTi systems with trained qSRO/MLPNet models are not
available, so these synthetic BCC alloys with random-initialised MLPs stand in for
them; see the paper's Sec. IV-B/IV-C for the originals):

* ``c1``  BCC 8^3 cells (1,024 sites), 4 species equiatomic, 12-input counts
          features (centre one-hot + shell-1/shell-2 species counts) -> 64 -> 64 -> 1,
          T = 1000 K, 100 sweeps.
* ``c2``  BCC 64^3 cells (524,288 sites), 4 species equiatomic, 108-input one-hot
          features (centre + 26 neighbours of shells 1-3) -> 128 -> 128 -> 1, T = 800 K.
* ``c3``  BCC 256^3 cells (33,554,432 sites), 5 species equiatomic, same 108-input
          model, T = 600 K.  One GPU's share of the paper's 1.009e9-atom
          strong-scaling system on 32 devices (Sec. V-B).
* ``c4``  96 replicas, cube edges uniform in 16..96 cells, 4 species with random
          compositions in [0.1, 0.4], temperatures log-spaced 300..3000 K.
* ``c5``  fit workload: 16^3-cell snapshots, 108-input model, labels from a seeded
          cluster-expansion Hamiltonian (``ce_params``), batches of 1,024 snapshots.
* ``fcc`` FCC 200^3 cells (32,000,000 sites, about one GPU's share of the paper's
          1.009e9-atom system on 32 devices), five species in the paper's
          Fe29Co29Ni28Al7Ti7 proportions (Sec. IV-C), the MLPNet shape of Eqs. (4)-(6)
          (76 one-hot inputs of the centre and its 18 shell-1/2 neighbours -> 96 -> 96
          -> 96 -> 1, ReLU) with random weights, T = 1000 K (the end of the paper's
          annealing schedule).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_LATTICE = 0
SEED_WEIGHTS = 1
SEED_PHILOX = 0
SEED_CE = 3
SEED_REPLICAS = 4
SEED_FD = 5

FEAT_COUNTS_S12 = 0   # 12 inputs: centre one-hot(4) + shell-1 counts(4) + shell-2 counts(4)
FEAT_ONEHOT_S123 = 1  # 108 inputs: one-hot(4) of the centre and of 26 neighbours (shells 1-3)

FEAT_QSRO_S123 = 2    # qSRO (Eq. 2) over shells 1-3
FEAT_FCC_MLPNET_S12 = 3  # FCC: one-hot(4) of the centre and 18 shell-1/2 neighbours, MLPNet

N_FEATURES = {FEAT_COUNTS_S12: 12, FEAT_ONEHOT_S123: 108}


def species_counts(n_sites: int, composition) -> np.ndarray:
    """Largest-remainder rounding of ``composition * n_sites`` (ties go to the lower species id)."""
    c = np.asarray(composition, dtype=np.float64)
    c = c / c.sum()
    exact = c * n_sites
    counts = np.floor(exact).astype(np.int64)
    rem = n_sites - int(counts.sum())
    frac = exact - counts
    # stable sort on -frac keeps species order among ties
    order = np.argsort(-frac, kind="stable")
    counts[order[:rem]] += 1
    return counts


def random_occupancy(cells, n_species: int = 4, composition=None, seed: int = SEED_LATTICE,
                     basis: int = 2) -> np.ndarray:
    """Uniformly random placement of a fixed composition on a lattice of ``cells`` cubic cells
    with ``basis`` sites per cell (2: BCC, 4: FCC).

    Returns uint8 species ids in canonical site order."""
    lx, ly, lz = (cells, cells, cells) if np.isscalar(cells) else cells
    n = int(basis) * int(lx) * int(ly) * int(lz)
    if composition is None:
        composition = np.full(n_species, 1.0 / n_species)
    counts = species_counts(n, composition)
    base = np.repeat(np.arange(len(counts), dtype=np.uint8), counts)
    return np.random.default_rng(seed).permutation(base).astype(np.uint8)


def mlp_param_sizes(n_in: int, hidden: int) -> list[tuple[str, tuple[int, ...], int]]:
    """(name, shape, fan_in) of W0, b0, W1, b1, W2, b2 in blob order (row-major [out][in])."""
    return [("W0", (hidden, n_in), n_in), ("b0", (hidden,), n_in),
            ("W1", (hidden, hidden), hidden), ("b1", (hidden,), hidden),
            ("W2", (1, hidden), hidden), ("b2", (1,), hidden)]


def mlp_n_params(n_in: int, hidden: int) -> int:
    return sum(int(np.prod(s)) for _, s, _ in mlp_param_sizes(n_in, hidden))


def mlp_params(n_in: int, hidden: int, seed: int = SEED_WEIGHTS, scale: float = 1.0) -> np.ndarray:
    """FP32 parameter blob, every entry ~ N(0, 1/fan_in) drawn in FP64 then rounded to FP32."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, shape, fan_in in mlp_param_sizes(n_in, hidden):
        parts.append(rng.normal(0.0, math.sqrt(1.0 / fan_in), size=shape).ravel())
    return (np.concatenate(parts) * scale).astype(np.float32)


def dirichlet_composition(rng: np.random.Generator, n_species: int = 4, lo: float = 0.1, hi: float = 0.4):
    while True:
        c = rng.dirichlet(np.ones(n_species))
        if np.all(c >= lo) and np.all(c <= hi):
            return c


@dataclass
class Workload:
    name: str
    cells: list                      # per replica: (Lx, Ly, Lz)
    n_species: int
    compositions: list               # per replica
    temperatures: list               # per replica, kelvin
    feature: int
    hidden: int
    sweeps: int
    seed: int = SEED_PHILOX
    extra: dict = field(default_factory=dict)
    lattice: str = "bcc"

    @property
    def basis(self) -> int:
        return 4 if self.lattice == "fcc" else 2

    @property
    def n_in(self) -> int:
        return FCC_N_INPUTS if self.lattice == "fcc" else N_FEATURES[self.feature]

    @property
    def sites(self) -> list:
        return [self.basis * a * b * c for a, b, c in self.cells]

    def occupancy(self) -> np.ndarray:
        """Concatenated per-replica occupancies (replica r drawn with seed SEED_LATTICE + r)."""
        parts = [random_occupancy(cl, self.n_species, comp, seed=SEED_LATTICE + r, basis=self.basis)
                 for r, (cl, comp) in enumerate(zip(self.cells, self.compositions))]
        return np.concatenate(parts)

    def params(self) -> np.ndarray:
        if self.lattice == "fcc":
            return mlpnet_params(self.hidden, SEED_WEIGHTS)
        return mlp_params(self.n_in, self.hidden, SEED_WEIGHTS)


def replica_set(n_replicas: int = 96, seed: int = SEED_REPLICAS, edge_lo: int = 16, edge_hi: int = 96):
    rng = np.random.default_rng(seed)
    edges = rng.integers(edge_lo, edge_hi + 1, size=n_replicas)
    comps = [dirichlet_composition(rng) for _ in range(n_replicas)]
    temps = [300.0 * 10.0 ** (r / (n_replicas - 1)) for r in range(n_replicas)]
    return [int(e) for e in edges], comps, temps


N_CE_TRIANGLES = 44  # distinct BCC triangle shapes with all three edges within shell 3


def ce_params(n_species: int = 4, n_items: int = 200, n_triangles: int = N_CE_TRIANGLES,
              seed: int = SEED_CE) -> dict:
    """Random draws of the reference cluster-expansion Hamiltonian.

    pair[m][p][q] = pair[m][q][p] ~ N(0, 0.03 eV) for shells m = 0..2 (drawn for p <= q in
    order m, p, q); then ``n_items`` distinct (triangle index, species triple) items, the
    triangle index uniform over the ``n_triangles`` canonical shapes (numbered in the
    lexicographic order of their canonical offsets) and each species uniform, duplicates
    redrawn; then J ~ N(0, 0.01 eV) per item."""
    rng = np.random.default_rng(seed)
    S = n_species
    pair = np.zeros((3, S, S))
    for m in range(3):
        for p in range(S):
            for q in range(p, S):
                pair[m, p, q] = pair[m, q, p] = rng.normal(0.0, 0.03)
    seen, tri, sp = set(), [], []
    while len(tri) < n_items:
        t = int(rng.integers(n_triangles))
        trip = tuple(int(v) for v in rng.integers(0, S, size=3))
        if (t, trip) in seen:
            continue
        seen.add((t, trip))
        tri.append(t)
        sp.append(trip)
    J = rng.normal(0.0, 0.01, size=n_items)
    return {"n_species": S, "pair": pair, "triangle": np.asarray(tri, dtype=np.int32),
            "species": np.asarray(sp, dtype=np.uint8), "J": J}


SEED_QSRO = 6

# The paper's alloy, Fe29Co29Ni28Al7Ti7 (Sec. IV-C), as species 0..4.
HEA_COMPOSITION = (0.29, 0.29, 0.28, 0.07, 0.07)
FCC_N_INPUTS = 76  # one-hot(4) of the centre and of the 18 shell-1/2 FCC neighbours


def mlpnet_param_sizes(hidden: int = 96, n_in: int = FCC_N_INPUTS):
    """(name, shape, fan_in) of the MLPNet blob (Eqs. (4)-(6)): W0, b0, W1, b1, W2, b2, W3, b3."""
    return [("W0", (hidden, n_in), n_in), ("b0", (hidden,), n_in),
            ("W1", (hidden, hidden), hidden), ("b1", (hidden,), hidden),
            ("W2", (hidden, hidden), hidden), ("b2", (hidden,), hidden),
            ("W3", (1, hidden), hidden), ("b3", (1,), hidden)]


def mlpnet_params(hidden: int = 96, seed: int = SEED_WEIGHTS, n_in: int = FCC_N_INPUTS) -> np.ndarray:
    """FP32 MLPNet blob, every entry ~ N(0, 1/fan_in) drawn in FP64 then rounded to FP32."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0.0, math.sqrt(1.0 / f), size=s).ravel() for _, s, f in mlpnet_param_sizes(hidden, n_in)]
    return np.concatenate(parts).astype(np.float32)


def qsro_params(n_species: int = 4, seed: int = SEED_QSRO) -> np.ndarray:
    """Synthetic qSRO coefficients (Eq. 2; trained ones are not available), FP32 blob
    [V[3][5][5], W[3][5], lambda, C]: V_m^{pp'} = V_m^{p'p} ~ N(0, 0.05 eV) for p' < p <
    n_species (drawn in order m, p, p'), W_m^p ~ N(0, 0.02 eV) for p < n_species, lambda =
    0.01, C = -0.1 eV; entries of absent species are zero."""
    rng = np.random.default_rng(seed)
    V = np.zeros((3, 5, 5))
    for m in range(3):
        for p in range(n_species):
            for q in range(p):
                V[m, p, q] = V[m, q, p] = rng.normal(0.0, 0.05)
    W = np.zeros((3, 5))
    W[:, :n_species] = rng.normal(0.0, 0.02, size=(3, n_species))
    return np.concatenate([V.ravel(), W.ravel(), [0.01, -0.1]]).astype(np.float32)


def snapshots(n: int, cells: int = 16, n_species: int = 4, seed: int = SEED_LATTICE + 100) -> np.ndarray:
    """``n`` snapshots (uint8 [n][2 cells^3]) with compositions drawn like the replica set
    (Dirichlet, every species in [0.1, 0.4]) and uniformly random placement."""
    rng = np.random.default_rng(seed)
    N = 2 * cells ** 3
    out = np.empty((n, N), dtype=np.uint8)
    for b in range(n):
        counts = species_counts(N, dirichlet_composition(rng, n_species))
        out[b] = rng.permutation(np.repeat(np.arange(n_species, dtype=np.uint8), counts))
    return out


def snapshot_temperatures(n: int, lo: float = 300.0, hi: float = 3000.0, seed: int = SEED_LATTICE + 101) -> np.ndarray:
    """Temperatures (K) of ``n`` snapshot chains, uniform on [lo, hi]."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n)


def workload(name: str, **over) -> Workload:
    name = name.lower()
    if name == "c1":
        w = Workload("c1", [(8, 8, 8)], 4, [None], [1000.0], FEAT_COUNTS_S12, 64, 100)
    elif name == "c2":
        w = Workload("c2", [(64, 64, 64)], 4, [None], [800.0], FEAT_ONEHOT_S123, 128, 1000)
    elif name == "c3":
        w = Workload("c3", [(256, 256, 256)], 5, [None], [600.0], FEAT_ONEHOT_S123, 128, 200)
    elif name == "c4":
        edges, comps, temps = replica_set()
        w = Workload("c4", [(e, e, e) for e in edges], 4, comps, temps, FEAT_ONEHOT_S123, 128, 500)
    elif name == "fcc":
        w = Workload("fcc", [(200, 200, 200)], 5, [HEA_COMPOSITION], [1000.0], FEAT_FCC_MLPNET_S12, 96, 100,
                     lattice="fcc")
    elif name == "c5":
        w = Workload("c5", [(16, 16, 16)], 4, [None], [1000.0], FEAT_ONEHOT_S123, 128, 0,
                     extra=dict(n_snapshots=65536, batch=1024))
    else:
        raise KeyError(name)
    for k, v in over.items():
        setattr(w, k, v)
    return w
