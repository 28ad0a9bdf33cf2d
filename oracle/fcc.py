"""FCC lattice of the oracle (``fcc_oracle.c``): geometry, the MLPNet of Eqs. (4)-(6) and the
qSRO model of Eq. (2) over FCC shells, zones, colouring and sweeps (test infrastructure only)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import Stats, TRIAL_DTYPE, TrialRec, ORDER_SNAPSHOT, _dims, _ptr, lib as _base_lib

MLPNET_S12, QSRO_S123 = 0, 1
N_INPUTS = 76
N_NBR = 42


class FccModel(C.Structure):
    _fields_ = [("model", C.c_int32), ("hidden", C.c_int32), ("params", C.POINTER(C.c_double))]


_ready = False


def lib():
    global _ready
    L = _base_lib()
    if not _ready:
        i32p, i64p, u8p, f64p = (C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                                 C.POINTER(C.c_uint8), C.POINTER(C.c_double))
        M = C.POINTER(FccModel)
        sig = {
            "or_fcc_n_sites": (C.c_int64, [i32p]),
            "or_fcc_site_pos": (None, [i32p, C.c_int64, i32p]),
            "or_fcc_site_at": (C.c_int64, [i32p, i32p]),
            "or_fcc_shell_table": (None, [i32p, i32p]),
            "or_fcc_neighbor": (C.c_int64, [i32p, C.c_int64, C.c_int32]),
            "or_fcc_n_params": (C.c_int64, [M]),
            "or_fcc_features": (None, [i32p, u8p, C.c_int64, C.c_int64, C.c_int64, f64p]),
            "or_fcc_mlpnet": (C.c_double, [M, f64p]),
            "or_fcc_site_energy": (C.c_double, [i32p, M, u8p, C.c_int64, C.c_int64, C.c_int64]),
            "or_fcc_all_site_energies": (None, [i32p, M, u8p, f64p]),
            "or_fcc_total_energy": (C.c_double, [i32p, M, u8p]),
            "or_fcc_omega": (C.c_int32, [i32p, C.c_int32, C.c_int64, C.c_int64, i64p]),
            "or_fcc_delta_e": (C.c_double, [i32p, M, u8p, C.c_int64, C.c_int64]),
            "or_fcc_n_colours": (C.c_int32, [i32p]),
            "or_fcc_colour_of": (C.c_int32, [i32p, C.c_int64]),
            "or_fcc_propose": (None, [C.c_uint64, C.c_int64, C.c_int64, C.c_int64, i32p, f64p]),
            "or_fcc_sweep": (C.c_int, [i32p, M, u8p, C.c_double, C.c_uint64, C.c_int64, C.c_int64,
                                       C.POINTER(Stats), C.c_void_p, C.c_int32, i64p, C.c_int32, C.c_int32,
                                       C.POINTER(C.c_int8)]),
            "or_fcc_warren_cowley": (None, [i32p, u8p, C.c_int32, f64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _ready = True
    return L


class MLPNet:
    """FP64 view of an FP32 MLPNet blob: W0[H][76], b0[H], W1[H][H], b1[H], W2[H][H], b2[H],
    W3[H], b3 (row-major [out][in])."""
    model = MLPNET_S12

    def __init__(self, hidden, params):
        self.hidden = int(hidden)
        self.params = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        want = n_params(hidden)
        if self.params.size != want:
            raise ValueError(f"MLPNet blob has {self.params.size} entries, expected {want}")
        self._c = FccModel(MLPNET_S12, self.hidden, _ptr(self.params, C.c_double))

    @property
    def c(self):
        return C.byref(self._c)


class QSRO:
    """FP64 view of a qSRO blob (Eq. 2) over FCC shells 1-3: V[3][5][5], W[3][5], lambda, C."""
    model = QSRO_S123
    hidden = 0

    def __init__(self, params):
        self.params = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        if self.params.size != 92:
            raise ValueError(f"qSRO blob has {self.params.size} entries, expected 92")
        self._c = FccModel(QSRO_S123, 0, _ptr(self.params, C.c_double))

    @property
    def c(self):
        return C.byref(self._c)


def n_params(hidden) -> int:
    H = int(hidden)
    return H * N_INPUTS + H + 2 * (H * H + H) + H + 1


def shell_table():
    off = np.zeros(3 * N_NBR, dtype=np.int32)
    sh = np.zeros(N_NBR, dtype=np.int32)
    lib().or_fcc_shell_table(_ptr(off, C.c_int32), _ptr(sh, C.c_int32))
    return off.reshape(N_NBR, 3), sh


def n_sites(cells) -> int:
    return int(lib().or_fcc_n_sites(_ptr(_dims(cells), C.c_int32)))


def site_pos(cells, s) -> np.ndarray:
    P = np.zeros(3, dtype=np.int32)
    lib().or_fcc_site_pos(_ptr(_dims(cells), C.c_int32), int(s), _ptr(P, C.c_int32))
    return P


def site_at(cells, P) -> int:
    P = np.ascontiguousarray(np.asarray(P, dtype=np.int32))
    return int(lib().or_fcc_site_at(_ptr(_dims(cells), C.c_int32), _ptr(P, C.c_int32)))


def neighbor(cells, s, k) -> int:
    return int(lib().or_fcc_neighbor(_ptr(_dims(cells), C.c_int32), int(s), int(k)))


def features(cells, occ, j, swap=(-1, -1)) -> np.ndarray:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    x = np.zeros(N_INPUTS, dtype=np.float64)
    lib().or_fcc_features(_ptr(_dims(cells), C.c_int32), _ptr(occ, C.c_uint8), int(j), int(swap[0]),
                          int(swap[1]), _ptr(x, C.c_double))
    return x


def mlpnet(model: MLPNet, x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().or_fcc_mlpnet(model.c, _ptr(x, C.c_double)))


def site_energy(cells, model, occ, j, swap=(-1, -1)) -> float:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    return float(lib().or_fcc_site_energy(_ptr(_dims(cells), C.c_int32), model.c, _ptr(occ, C.c_uint8),
                                          int(j), int(swap[0]), int(swap[1])))


def all_site_energies(cells, model, occ) -> np.ndarray:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    e = np.zeros(occ.size, dtype=np.float64)
    lib().or_fcc_all_site_energies(_ptr(_dims(cells), C.c_int32), model.c, _ptr(occ, C.c_uint8),
                                   _ptr(e, C.c_double))
    return e


def total_energy(cells, model, occ) -> float:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    return float(lib().or_fcc_total_energy(_ptr(_dims(cells), C.c_int32), model.c, _ptr(occ, C.c_uint8)))


def omega(cells, model_kind, i, n) -> np.ndarray:
    out = np.zeros(2 + 2 * N_NBR, dtype=np.int64)
    k = lib().or_fcc_omega(_ptr(_dims(cells), C.c_int32), int(model_kind), int(i), int(n), _ptr(out, C.c_int64))
    return out[:k].copy()


def delta_e(cells, model, occ, i, n) -> float:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    return float(lib().or_fcc_delta_e(_ptr(_dims(cells), C.c_int32), model.c, _ptr(occ, C.c_uint8),
                                      int(i), int(n)))


def n_colours(cells) -> int:
    return int(lib().or_fcc_n_colours(_ptr(_dims(cells), C.c_int32)))


def colours(cells) -> np.ndarray:
    d = _dims(cells)
    f = lib().or_fcc_colour_of
    dp = _ptr(d, C.c_int32)
    return np.array([f(dp, s) for s in range(n_sites(cells))], dtype=np.int32)


def propose(seed, site, sweep, replica):
    d = C.c_int32()
    u = C.c_double()
    lib().or_fcc_propose(seed, site, sweep, replica, C.byref(d), C.byref(u))
    return d.value, u.value


def sweep(cells, model, occ: np.ndarray, temperature_K: float, seed: int, replica: int, sweep_index: int,
          stats: Stats | None = None, trace: bool = False, order: int = ORDER_SNAPSHOT, given_order=None,
          nthreads: int = 1, colours_limit: int = -1, force=None):
    """Advance ``occ`` (uint8, modified in place) by one sweep; returns (stats, trace|None).
    force (optional int8 [N]): 0/1 replaces the decision of the different-species trial at
    that site, -1 keeps the Metropolis decision."""
    assert occ.dtype == np.uint8 and occ.flags.c_contiguous
    st = stats if stats is not None else Stats()
    tr = np.zeros(occ.size, dtype=TRIAL_DTYPE) if trace else None
    go = None if given_order is None else np.ascontiguousarray(given_order, dtype=np.int64)
    fo = None if force is None else np.ascontiguousarray(force, dtype=np.int8)
    assert fo is None or fo.size == occ.size
    rc = lib().or_fcc_sweep(_ptr(_dims(cells), C.c_int32), model.c, _ptr(occ, C.c_uint8), float(temperature_K),
                            int(seed), int(replica), int(sweep_index), C.byref(st),
                            tr.ctypes.data if tr is not None else None, order,
                            _ptr(go, C.c_int64) if go is not None else None, nthreads, colours_limit,
                            _ptr(fo, C.c_int8) if fo is not None else None)
    if rc != 0:
        raise MemoryError("oracle sweep failed to allocate")
    return st, tr


def warren_cowley(cells, occ, n_species) -> np.ndarray:
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    a = np.zeros((3, n_species, n_species), dtype=np.float64)
    lib().or_fcc_warren_cowley(_ptr(_dims(cells), C.c_int32), _ptr(occ, C.c_uint8), n_species,
                               _ptr(a, C.c_double))
    return a
