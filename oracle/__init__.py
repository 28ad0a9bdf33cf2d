"""Python view of the plain CPU oracle (test infrastructure only).

The oracle is the slow FP64 C library in ``smc_oracle.c`` (BCC), ``fcc_oracle.c`` (FCC, see
``oracle.fcc``) and ``fit_oracle.c`` (the fit).  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import this package; the
product package never does.  ``build()`` compiles the library with gcc.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "smc_oracle.c")
SOURCES = [SRC, os.path.join(HERE, "fit_oracle.c"), os.path.join(HERE, "fcc_oracle.c")]
LIB = os.path.join(HERE, "liboracle.so")

FEAT_COUNTS_S12, FEAT_ONEHOT_S123, FEAT_QSRO_S123 = 0, 1, 2
ACT_SILU, ACT_IDENTITY, ACT_RELU, ACT_SQUARE = 0, 1, 2, 3
ORDER_SNAPSHOT, ORDER_FORWARD, ORDER_REVERSE, ORDER_GIVEN = 0, 1, 2, 3
KB_EV_PER_K = 8.617333262e-5


def build(force: bool = True) -> str:
    stale = not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(f) for f in SOURCES)
    if force or stale:
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-Wno-unused-parameter",
                               *SOURCES, "-o", LIB + ".tmp", "-lm"], cwd=HERE)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Model(C.Structure):
    _fields_ = [("feature", C.c_int32), ("hidden", C.c_int32), ("act0", C.c_int32),
                ("act1", C.c_int32), ("params", C.POINTER(C.c_double))]


class CE(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("pair", C.POINTER(C.c_double)), ("n_items", C.c_int32),
                ("offsets", C.POINTER(C.c_int32)), ("species", C.POINTER(C.c_uint8)),
                ("J", C.POINTER(C.c_double))]


class TrialRec(C.Structure):
    _fields_ = [("site", C.c_int64), ("partner", C.c_int64), ("dE", C.c_double),
                ("theta", C.c_double), ("u", C.c_double), ("dir", C.c_int32),
                ("same", C.c_int32), ("accept", C.c_int32), ("colour", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("attempts", C.c_uint64), ("diff_species", C.c_uint64),
                ("accepts", C.c_uint64), ("e_run", C.c_double)]


TRIAL_DTYPE = np.dtype([("site", np.int64), ("partner", np.int64), ("dE", np.float64),
                        ("theta", np.float64), ("u", np.float64), ("dir", np.int32),
                        ("same", np.int32), ("accept", np.int32), ("colour", np.int32)])
assert TRIAL_DTYPE.itemsize == C.sizeof(TrialRec)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        i32p, i64p, u8p, f64p = (C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_uint8), C.POINTER(C.c_double))
        u64p = C.POINTER(C.c_uint64)
        sig = {
            "or_philox4x64_10": (None, [u64p, u64p, u64p]),
            "or_n_sites": (C.c_int64, [i32p]),
            "or_site_pos": (None, [i32p, C.c_int64, i32p]),
            "or_site_at": (C.c_int64, [i32p, i32p]),
            "or_shell_table": (None, [i32p, i32p]),
            "or_neighbor": (C.c_int64, [i32p, C.c_int64, C.c_int32]),
            "or_n_inputs": (C.c_int32, [C.c_int32]),
            "or_features": (None, [i32p, C.c_int32, u8p, C.c_int64, C.c_int64, C.c_int64, f64p]),
            "or_mlp": (C.c_double, [C.POINTER(Model), f64p]),
            "or_site_energy": (C.c_double, [i32p, C.POINTER(Model), u8p, C.c_int64, C.c_int64,
                                            C.c_int64]),
            "or_total_energy": (C.c_double, [i32p, C.POINTER(Model), u8p]),
            "or_all_site_energies": (None, [i32p, C.POINTER(Model), u8p, f64p]),
            "or_omega": (C.c_int32, [i32p, C.c_int32, C.c_int64, C.c_int64, i64p]),
            "or_delta_e": (C.c_double, [i32p, C.POINTER(Model), u8p, C.c_int64, C.c_int64]),
            "or_n_colours": (C.c_int32, [i32p]),
            "or_colour_of": (C.c_int32, [i32p, C.c_int64]),
            "or_propose": (None, [C.c_uint64, C.c_int64, C.c_int64, C.c_int64, i32p, f64p]),
            "or_theta": (C.c_double, [C.c_double, C.c_double]),
            "or_accept": (C.c_int32, [C.c_double, C.c_double]),
            "or_trial": (None, [i32p, C.POINTER(Model), u8p, C.c_double, C.c_uint64, C.c_int64,
                                C.c_int64, C.c_int64, C.POINTER(TrialRec)]),
            "or_sweep": (C.c_int, [i32p, C.POINTER(Model), u8p, C.c_double, C.c_uint64, C.c_int64,
                                   C.c_int64, C.POINTER(Stats), C.c_void_p, C.c_int32, i64p,
                                   C.c_int32, C.c_int32, C.POINTER(C.c_int8)]),
            "or_proposals": (None, [i32p, C.c_uint64, C.c_int64, C.c_int64, C.c_double, i64p, C.c_int64,
                                    i32p, i64p, f64p]),
            "or_warren_cowley": (None, [i32p, u8p, C.c_int32, f64p]),
            "or_ce_triangles": (C.c_int32, [i32p, C.c_int32]),
            "or_ce_site_energy": (C.c_double, [i32p, C.POINTER(CE), u8p, C.c_int64]),
            "or_ce_total_local": (C.c_double, [i32p, C.POINTER(CE), u8p]),
            "or_ce_total_brute": (C.c_double, [i32p, C.POINTER(CE), u8p]),
            "or_n_params": (C.c_int64, [C.POINTER(Model)]),
            "or_energy_grad": (None, [i32p, C.POINTER(Model), u8p, C.c_int32, f64p, f64p, f64p, C.c_int32]),
            "or_fit_loss_grad": (C.c_double, [i32p, C.POINTER(Model), u8p, C.c_int32, f64p, f64p, f64p,
                                              C.c_int32]),
            "or_fit_fd": (None, [i32p, C.POINTER(Model), u8p, C.c_int32, f64p, i64p, C.c_int32, C.c_double,
                                 f64p, C.c_int32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def _dims(cells) -> np.ndarray:
    if np.isscalar(cells):
        cells = (cells, cells, cells)
    return np.ascontiguousarray(np.asarray(cells, dtype=np.int32))


@dataclass
class MLP:
    """FP64 view of an FP32 parameter blob (W0, b0, W1, b1, W2, b2; row-major [out][in])."""
    feature: int
    hidden: int
    params: np.ndarray
    act0: int = ACT_SILU
    act1: int = ACT_SILU

    def __post_init__(self):
        self.params = np.ascontiguousarray(np.asarray(self.params, dtype=np.float64))
        n_in = 12 if self.feature == FEAT_COUNTS_S12 else 108
        H = self.hidden
        want = H * n_in + H + H * H + H + H + 1
        if self.params.size != want:
            raise ValueError(f"parameter blob has {self.params.size} entries, expected {want}")
        self._c = Model(self.feature, self.hidden, self.act0, self.act1,
                        _ptr(self.params, C.c_double))

    @property
    def c(self):
        return C.byref(self._c)

    @property
    def n_in(self) -> int:
        return 12 if self.feature == FEAT_COUNTS_S12 else 108


class QSRO:
    """FP64 view of a qSRO parameter blob (Eq. 2): V[3][5][5] (symmetric), W[3][5], lambda, C."""

    feature = FEAT_QSRO_S123
    hidden = 0

    def __init__(self, params):
        self.params = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        if self.params.size != 92:
            raise ValueError(f"qSRO blob has {self.params.size} entries, expected 92")
        self._c = Model(FEAT_QSRO_S123, 0, 0, 0, _ptr(self.params, C.c_double))

    @property
    def c(self):
        return C.byref(self._c)


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(out, C.c_uint64))
    return out


def shell_table():
    off = np.zeros(78, dtype=np.int32)
    sh = np.zeros(26, dtype=np.int32)
    lib().or_shell_table(_ptr(off, C.c_int32), _ptr(sh, C.c_int32))
    return off.reshape(26, 3), sh


def n_sites(cells) -> int:
    return int(lib().or_n_sites(_ptr(_dims(cells), C.c_int32)))


def site_pos(cells, s) -> np.ndarray:
    P = np.zeros(3, dtype=np.int32)
    lib().or_site_pos(_ptr(_dims(cells), C.c_int32), int(s), _ptr(P, C.c_int32))
    return P


def neighbor(cells, s, k) -> int:
    return int(lib().or_neighbor(_ptr(_dims(cells), C.c_int32), int(s), int(k)))


def features(cells, feature, occ, j, swap=(-1, -1)) -> np.ndarray:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    x = np.zeros(12 if feature == FEAT_COUNTS_S12 else 108, dtype=np.float64)
    lib().or_features(_ptr(_dims(cells), C.c_int32), feature, _ptr(occ, C.c_uint8), int(j),
                      int(swap[0]), int(swap[1]), _ptr(x, C.c_double))
    return x


def mlp(model: MLP, x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().or_mlp(model.c, _ptr(x, C.c_double)))


def site_energy(cells, model: MLP, occ, j, swap=(-1, -1)) -> float:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    return float(lib().or_site_energy(_ptr(_dims(cells), C.c_int32), model.c, _ptr(occ, C.c_uint8),
                                      int(j), int(swap[0]), int(swap[1])))


def total_energy(cells, model: MLP, occ) -> float:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    return float(lib().or_total_energy(_ptr(_dims(cells), C.c_int32), model.c,
                                       _ptr(occ, C.c_uint8)))


def all_site_energies(cells, model: MLP, occ) -> np.ndarray:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    e = np.zeros(occ.size, dtype=np.float64)
    lib().or_all_site_energies(_ptr(_dims(cells), C.c_int32), model.c, _ptr(occ, C.c_uint8),
                               _ptr(e, C.c_double))
    return e


def omega(cells, feature, i, n) -> np.ndarray:
    out = np.zeros(54, dtype=np.int64)
    k = lib().or_omega(_ptr(_dims(cells), C.c_int32), feature, int(i), int(n), _ptr(out, C.c_int64))
    return out[:k].copy()


def delta_e(cells, model: MLP, occ, i, n) -> float:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    return float(lib().or_delta_e(_ptr(_dims(cells), C.c_int32), model.c, _ptr(occ, C.c_uint8),
                                  int(i), int(n)))


def n_colours(cells) -> int:
    return int(lib().or_n_colours(_ptr(_dims(cells), C.c_int32)))


def colours(cells) -> np.ndarray:
    d = _dims(cells)
    n = n_sites(cells)
    f = lib().or_colour_of
    dp = _ptr(d, C.c_int32)
    return np.array([f(dp, s) for s in range(n)], dtype=np.int32)


def propose(seed, site, sweep, replica):
    d = C.c_int32()
    u = C.c_double()
    lib().or_propose(seed, site, sweep, replica, C.byref(d), C.byref(u))
    return d.value, u.value


def proposals(cells, seed, replica, sweep_index, temperature_K, sites):
    """(partner slot, partner site, theta) of many trial sites at once."""
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    n = sites.size
    d = np.zeros(n, dtype=np.int32)
    p = np.zeros(n, dtype=np.int64)
    th = np.zeros(n, dtype=np.float64)
    lib().or_proposals(_ptr(_dims(cells), C.c_int32), int(seed), int(replica), int(sweep_index),
                       float(temperature_K), _ptr(sites, C.c_int64), n, _ptr(d, C.c_int32),
                       _ptr(p, C.c_int64), _ptr(th, C.c_double))
    return d, p, th


def theta(temperature_K, u) -> float:
    return float(lib().or_theta(temperature_K, u))


def trial(cells, model: MLP, occ, temperature_K, seed, replica, sweep, site) -> np.void:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    rec = np.zeros(1, dtype=TRIAL_DTYPE)
    lib().or_trial(_ptr(_dims(cells), C.c_int32), model.c, _ptr(occ, C.c_uint8), temperature_K,
                   seed, replica, sweep, site, rec.ctypes.data_as(C.POINTER(TrialRec)))
    return rec[0]


def sweep(cells, model: MLP, occ: np.ndarray, temperature_K: float, seed: int, replica: int,
          sweep_index: int, stats: Stats | None = None, trace: bool = False,
          order: int = ORDER_SNAPSHOT, given_order=None, nthreads: int = 1,
          colours_limit: int = -1, force=None):
    """Advance ``occ`` (uint8, modified in place) by one sweep; returns (stats, trace|None).

    force (optional int8 [N]): 0/1 replaces the decision of the different-species trial at
    that site, -1 keeps the Metropolis decision."""
    assert occ.dtype == np.uint8 and occ.flags.c_contiguous
    st = stats if stats is not None else Stats()
    tr = np.zeros(occ.size, dtype=TRIAL_DTYPE) if trace else None
    go = None
    if given_order is not None:
        go = np.ascontiguousarray(given_order, dtype=np.int64)
    fo = None
    if force is not None:
        fo = np.ascontiguousarray(force, dtype=np.int8)
        assert fo.size == occ.size
    rc = lib().or_sweep(_ptr(_dims(cells), C.c_int32), model.c, _ptr(occ, C.c_uint8),
                        float(temperature_K), int(seed), int(replica), int(sweep_index),
                        C.byref(st), tr.ctypes.data if tr is not None else None, order,
                        _ptr(go, C.c_int64) if go is not None else None, nthreads, colours_limit,
                        _ptr(fo, C.c_int8) if fo is not None else None)
    if rc != 0:
        raise MemoryError("oracle sweep failed to allocate")
    return st, tr


def warren_cowley(cells, occ, n_species) -> np.ndarray:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    a = np.zeros((3, n_species, n_species), dtype=np.float64)
    lib().or_warren_cowley(_ptr(_dims(cells), C.c_int32), _ptr(occ, C.c_uint8), n_species,
                           _ptr(a, C.c_double))
    return a


# ---------------------------------------------------------------- differentiation pattern

class CEModel:
    """FP64 view of a cluster-expansion Hamiltonian: pair[3][S][S], and items of
    (canonical triangle offsets [6], species triple [3], J)."""

    def __init__(self, n_species, pair, offsets, species, J):
        self.n_species = int(n_species)
        self.pair = np.ascontiguousarray(np.asarray(pair, dtype=np.float64).reshape(3, n_species, n_species))
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 6))
        self.species = np.ascontiguousarray(np.asarray(species, dtype=np.uint8).reshape(-1, 3))
        self.J = np.ascontiguousarray(np.asarray(J, dtype=np.float64).reshape(-1))
        self._c = CE(self.n_species, _ptr(self.pair, C.c_double), len(self.J), _ptr(self.offsets, C.c_int32),
                     _ptr(self.species, C.c_uint8), _ptr(self.J, C.c_double))

    @property
    def c(self):
        return C.byref(self._c)


def ce_triangles() -> np.ndarray:
    out = np.zeros((1024, 6), dtype=np.int32)
    n = lib().or_ce_triangles(_ptr(out, C.c_int32), 1024)
    return out[:n].copy()


def ce_site_energy(cells, ce: CEModel, occ, s) -> float:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    return float(lib().or_ce_site_energy(_ptr(_dims(cells), C.c_int32), ce.c, _ptr(occ, C.c_uint8), int(s)))


def ce_total(cells, ce: CEModel, occ, brute=False) -> float:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    f = lib().or_ce_total_brute if brute else lib().or_ce_total_local
    return float(f(_ptr(_dims(cells), C.c_int32), ce.c, _ptr(occ, C.c_uint8)))


def snapshot_energies(cells, model: MLP, snaps, nthreads=8) -> np.ndarray:
    snaps = np.ascontiguousarray(snaps, dtype=np.uint8)
    B = snaps.shape[0]
    S = np.zeros(B)
    lib().or_energy_grad(_ptr(_dims(cells), C.c_int32), model.c, _ptr(snaps, C.c_uint8), B,
                         _ptr(S, C.c_double), None, None, nthreads)
    return S


def energy_grad(cells, model: MLP, snaps, gE, nthreads=8) -> np.ndarray:
    """sum_b gE[b] dS_b/dparams (FP64)."""
    snaps = np.ascontiguousarray(snaps, dtype=np.uint8)
    gE = np.ascontiguousarray(gE, dtype=np.float64)
    g = np.zeros(model.params.size)
    lib().or_energy_grad(_ptr(_dims(cells), C.c_int32), model.c, _ptr(snaps, C.c_uint8), snaps.shape[0],
                         None, _ptr(gE, C.c_double), _ptr(g, C.c_double), nthreads)
    return g


def fit_loss_grad(cells, model: MLP, snaps, labels, nthreads=8, want_grad=True):
    """(loss, S[batch], grad|None) of loss = mean_b ((S_b - E_b)/N)^2."""
    snaps = np.ascontiguousarray(snaps, dtype=np.uint8)
    labels = np.ascontiguousarray(labels, dtype=np.float64)
    B = snaps.shape[0]
    S = np.zeros(B)
    g = np.zeros(model.params.size) if want_grad else None
    loss = lib().or_fit_loss_grad(_ptr(_dims(cells), C.c_int32), model.c, _ptr(snaps, C.c_uint8), B,
                                  _ptr(labels, C.c_double), _ptr(S, C.c_double),
                                  _ptr(g, C.c_double) if g is not None else None, nthreads)
    return float(loss), S, g


def fit_fd(cells, model: MLP, snaps, labels, idx, h=1e-6, nthreads=8) -> np.ndarray:
    snaps = np.ascontiguousarray(snaps, dtype=np.uint8)
    labels = np.ascontiguousarray(labels, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(idx.size)
    lib().or_fit_fd(_ptr(_dims(cells), C.c_int32), model.c, _ptr(snaps, C.c_uint8), snaps.shape[0],
                    _ptr(labels, C.c_double), _ptr(idx, C.c_int64), idx.size, float(h), _ptr(out, C.c_double),
                    nthreads)
    return out
