"""ctypes binding of libsmc.so (argument marshalling only; every step runs in HIP kernels).

The functions here carry the names of the C ABI in ``include/smc.h`` and take raw device
pointers (ints) and host numpy arrays.  There is no fallback: if the library is not built
or cannot be loaded, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsmc.so")

SMC_OK, SMC_E_INVALID, SMC_E_UNSUPPORTED, SMC_E_DEVICE, SMC_E_STATE, SMC_E_NOMEM = 0, -1, -2, -3, -4, -5
SMC_FP32, SMC_BF16, SMC_BF16X3, SMC_FP8_E4M3, SMC_FP64 = 0, 1, 2, 3, 4
SMC_FEAT_COUNTS_S12, SMC_FEAT_ONEHOT_S123, SMC_FEAT_QSRO_S123, SMC_FEAT_MLPNET_S12 = 0, 1, 2, 3
SMC_LATTICE_BCC, SMC_LATTICE_FCC = 0, 1
LATTICES = {"bcc": SMC_LATTICE_BCC, "fcc": SMC_LATTICE_FCC}
BASIS = {SMC_LATTICE_BCC: 2, SMC_LATTICE_FCC: 4}

PRECISIONS = {"fp32": SMC_FP32, "bf16": SMC_BF16, "bf16x3": SMC_BF16X3, "fp8": SMC_FP8_E4M3,
              "fp64": SMC_FP64}

EXPORTS = ["smc_init", "smc_sweep", "smc_energy", "smc_site_energies", "smc_set_params",
           "smc_refresh", "smc_counters", "smc_delta_e64", "smc_delta_e64_noalloc", "smc_profile", "smc_kernel_times", "smc_get_sweep",
           "smc_set_sweep", "smc_set_temperatures", "smc_warren_cowley", "smc_set_strategy", "smc_get_strategy", "smc_use_graph", "smc_set_variant", "smc_get_variant", "smc_autotune",
           "smc_energy_fwd", "smc_energy_bwd", "smc_fit_step", "smc_ce_energy", "smc_ce_triangles", "smc_lattice_shells",
           "smc_n_sites", "smc_n_colours", "smc_destroy", "smc_last_error", "smc_status_string"]


class smc_config(C.Structure):
    _fields_ = [("n_replicas", C.c_int32), ("cells", C.POINTER(C.c_int32)),
                ("temperature_K", C.POINTER(C.c_double)), ("n_species", C.c_int32),
                ("feature", C.c_int32), ("hidden", C.c_int32), ("precision", C.c_int32),
                ("seed", C.c_uint64), ("guard_eV", C.c_double), ("lattice", C.c_int32)]


class smc_stats(C.Structure):
    _fields_ = [("attempts", C.POINTER(C.c_uint64)), ("diff_species", C.POINTER(C.c_uint64)),
                ("accepts", C.POINTER(C.c_uint64)), ("rechecks", C.POINTER(C.c_uint64)),
                ("trace_dE", C.c_void_p), ("trace_dE_fast", C.c_void_p),
                ("trace_flags", C.c_void_p)]


class smc_ce(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("pair", C.POINTER(C.c_double)), ("n_items", C.c_int32),
                ("triangle", C.POINTER(C.c_int32)), ("species", C.POINTER(C.c_uint8)),
                ("J", C.POINTER(C.c_double))]


class SMCError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libsmc.so (raises if it is missing: there is no other implementation)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SMCError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        sig = {
            "smc_init": (C.c_int, [C.POINTER(smc_config), vp, vp, vp, vp, C.POINTER(vp)]),
            "smc_sweep": (C.c_int, [vp, C.c_int32, C.POINTER(smc_stats)]),
            "smc_energy": (C.c_int, [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
            "smc_site_energies": (C.c_int, [vp, C.c_int32, vp]),
            "smc_set_params": (C.c_int, [vp, vp]),
            "smc_refresh": (C.c_int, [vp]),
            "smc_counters": (C.c_int, [vp, C.POINTER(C.c_uint64), C.c_int32]),
            "smc_delta_e64": (C.c_int, [vp, C.c_int32, C.c_uint64, C.POINTER(C.c_int64), C.c_int32,
                                        C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
            "smc_delta_e64_noalloc": (C.c_int, [vp, C.c_int32, C.c_uint64, vp, C.c_int32, vp, vp]),
            "smc_profile": (C.c_int, [vp, C.c_int32]),
            "smc_kernel_times": (C.c_int, [vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                           C.POINTER(C.c_int64)]),
            "smc_get_sweep": (C.c_int, [vp, C.POINTER(C.c_uint64)]),
            "smc_set_sweep": (C.c_int, [vp, C.c_uint64]),
            "smc_set_temperatures": (C.c_int, [vp, C.POINTER(C.c_double)]),
            "smc_warren_cowley": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_double)]),
            "smc_set_strategy": (C.c_int, [vp, C.c_int32]),
            "smc_get_strategy": (C.c_int, [vp, C.POINTER(C.c_int32)]),
            "smc_use_graph": (C.c_int, [vp, C.c_int32]),
            "smc_set_variant": (C.c_int, [vp, C.c_int32]),
            "smc_get_variant": (C.c_int, [vp, C.POINTER(C.c_int32)]),
            "smc_autotune": (C.c_int, [vp, C.c_char_p, C.POINTER(C.c_int32), C.POINTER(C.c_float)]),
            "smc_energy_fwd": (C.c_int, [vp, vp, C.c_int32, C.c_int32, vp, vp]),
            "smc_energy_bwd": (C.c_int, [vp, vp, C.c_int32, C.c_int32, vp, vp, vp]),
            "smc_fit_step": (C.c_int, [vp, vp, C.c_int32, C.c_int32, vp, vp, vp, vp, C.c_float, C.c_int32,
                                       C.POINTER(C.c_double)]),
            "smc_ce_energy": (C.c_int, [vp, C.POINTER(smc_ce), vp, C.c_int32, C.c_int32, vp]),
            "smc_ce_triangles": (C.c_int, [C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]),
            "smc_lattice_shells": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32]),
            "smc_n_sites": (C.c_int, [vp, C.POINTER(C.c_int64)]),
            "smc_n_colours": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_int32)]),
            "smc_destroy": (None, [vp]),
            "smc_last_error": (C.c_char_p, [vp]),
            "smc_status_string": (C.c_char_p, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int, ctx=None):
    if rc != SMC_OK:
        msg = lib().smc_status_string(rc).decode()
        if ctx:
            msg += ": " + lib().smc_last_error(ctx).decode()
        raise SMCError(f"libsmc returned {rc} ({msg})")


def _u64(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_uint64))


def smc_init(cells, temperatures, n_species, feature, hidden, precision, seed, guard_eV,
             occ_ptr, params_ptr, ecache_ptr, stream_ptr, lattice=SMC_LATTICE_BCC):
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, 3))
    temps = np.ascontiguousarray(np.asarray(temperatures, dtype=np.float64).reshape(-1))
    cfg = smc_config(len(temps), cells.ctypes.data_as(C.POINTER(C.c_int32)),
                     temps.ctypes.data_as(C.POINTER(C.c_double)), n_species, feature, hidden,
                     precision, seed, guard_eV, lattice)
    ctx = C.c_void_p()
    rc = lib().smc_init(C.byref(cfg), occ_ptr, params_ptr, ecache_ptr, stream_ptr, C.byref(ctx))
    check(rc)
    return ctx.value


def smc_sweep(ctx, n_sweeps, attempts=None, diff_species=None, accepts=None, rechecks=None,
              trace_dE=0, trace_dE_fast=0, trace_flags=0, with_stats=False):
    st = None
    if with_stats:
        st = smc_stats(_u64(attempts), _u64(diff_species), _u64(accepts), _u64(rechecks),
                       trace_dE or None, trace_dE_fast or None, trace_flags or None)
    check(lib().smc_sweep(ctx, n_sweeps, C.byref(st) if st is not None else None), ctx)


def smc_energy(ctx, n_replicas):
    es = np.zeros(n_replicas)
    er = np.zeros(n_replicas)
    check(lib().smc_energy(ctx, es.ctypes.data_as(C.POINTER(C.c_double)),
                           er.ctypes.data_as(C.POINTER(C.c_double))), ctx)
    return es, er


def smc_site_energies(ctx, precision, out_ptr):
    check(lib().smc_site_energies(ctx, precision, out_ptr), ctx)


def smc_set_params(ctx, params_ptr):
    check(lib().smc_set_params(ctx, params_ptr), ctx)


def smc_refresh(ctx):
    check(lib().smc_refresh(ctx), ctx)


def smc_counters(ctx, n_replicas, reset=False):
    out = np.zeros((4, n_replicas), dtype=np.uint64)
    check(lib().smc_counters(ctx, out.ctypes.data_as(C.POINTER(C.c_uint64)), int(reset)), ctx)
    return out


def smc_delta_e64(ctx, replica, sweep, sites):
    sites = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    partner = np.zeros(sites.size, dtype=np.int64)
    dE = np.zeros(sites.size, dtype=np.float64)
    check(lib().smc_delta_e64(ctx, replica, sweep, sites.ctypes.data_as(C.POINTER(C.c_int64)), sites.size,
                              partner.ctypes.data_as(C.POINTER(C.c_int64)),
                              dE.ctypes.data_as(C.POINTER(C.c_double))), ctx)
    return partner, dE


def smc_delta_e64_noalloc(ctx, replica, sweep, sites_ptr, n, partner_ptr, dE_ptr):
    """Device pointers (ints); asynchronous, allocates nothing."""
    check(lib().smc_delta_e64_noalloc(ctx, int(replica), int(sweep), sites_ptr or None, int(n),
                                      partner_ptr or None, dE_ptr or None), ctx)


def smc_profile(ctx, enable):
    check(lib().smc_profile(ctx, int(bool(enable))), ctx)


def smc_kernel_times(ctx):
    a, b, n = C.c_double(), C.c_double(), C.c_int64()
    check(lib().smc_kernel_times(ctx, C.byref(a), C.byref(b), C.byref(n)), ctx)
    return a.value, b.value, n.value


def smc_get_sweep(ctx) -> int:
    s = C.c_uint64()
    check(lib().smc_get_sweep(ctx, C.byref(s)), ctx)
    return s.value


def smc_set_sweep(ctx, sweep):
    check(lib().smc_set_sweep(ctx, sweep), ctx)


def smc_lattice_shells(lattice):
    """(offsets [k][3], shells [k]) of the neighbour slots of a lattice, in slot order."""
    off = np.zeros((64, 3), dtype=np.int32)
    sh = np.zeros(64, dtype=np.int32)
    n = lib().smc_lattice_shells(int(lattice), off.ctypes.data_as(C.POINTER(C.c_int32)),
                                 sh.ctypes.data_as(C.POINTER(C.c_int32)), 64)
    if n < 0:
        check(n)
    return off[:n].copy(), sh[:n].copy()


def smc_set_temperatures(ctx, temperatures):
    t = np.ascontiguousarray(np.asarray(temperatures, dtype=np.float64).reshape(-1))
    check(lib().smc_set_temperatures(ctx, t.ctypes.data_as(C.POINTER(C.c_double))), ctx)


def smc_warren_cowley(ctx, replica, n_species):
    a = np.zeros((3, n_species, n_species), dtype=np.float64)
    check(lib().smc_warren_cowley(ctx, int(replica), a.ctypes.data_as(C.POINTER(C.c_double))), ctx)
    return a


SMC_STRATEGY_ZONE, SMC_STRATEGY_DOUBLE_LATTICE = 0, 1
STRATEGIES = {"zone": SMC_STRATEGY_ZONE, "double_lattice": SMC_STRATEGY_DOUBLE_LATTICE}


def smc_set_strategy(ctx, strategy):
    check(lib().smc_set_strategy(ctx, int(strategy)), ctx)


def smc_get_strategy(ctx) -> int:
    v = C.c_int32()
    check(lib().smc_get_strategy(ctx, C.byref(v)), ctx)
    return v.value


def smc_use_graph(ctx, enable):
    check(lib().smc_use_graph(ctx, int(bool(enable))), ctx)


def smc_set_variant(ctx, variant):
    check(lib().smc_set_variant(ctx, int(variant)), ctx)


def smc_get_variant(ctx) -> int:
    v = C.c_int32()
    check(lib().smc_get_variant(ctx, C.byref(v)), ctx)
    return v.value


def smc_autotune(ctx, cache_path=None):
    chosen = C.c_int32()
    ms = np.zeros(4, dtype=np.float32)
    check(lib().smc_autotune(ctx, cache_path.encode() if cache_path else None, C.byref(chosen),
                             ms.ctypes.data_as(C.POINTER(C.c_float))), ctx)
    return chosen.value, ms


def smc_energy_fwd(ctx, snap_ptr, batch, cells_per_axis, params_ptr, e_out_ptr):
    check(lib().smc_energy_fwd(ctx, snap_ptr, batch, cells_per_axis, params_ptr, e_out_ptr), ctx)


def smc_energy_bwd(ctx, snap_ptr, batch, cells_per_axis, params_ptr, grad_e_ptr, grad_params_ptr):
    check(lib().smc_energy_bwd(ctx, snap_ptr, batch, cells_per_axis, params_ptr, grad_e_ptr, grad_params_ptr), ctx)


def smc_fit_step(ctx, snap_ptr, batch, cells_per_axis, label_ptr, params_ptr, m_ptr, v_ptr, lr, step,
                 want_loss=True):
    loss = C.c_double(float("nan"))
    check(lib().smc_fit_step(ctx, snap_ptr, batch, cells_per_axis, label_ptr, params_ptr, m_ptr, v_ptr, lr, step,
                             C.byref(loss) if want_loss else None), ctx)
    return loss.value if want_loss else None


def smc_ce_triangles() -> np.ndarray:
    n = C.c_int32()
    check(lib().smc_ce_triangles(None, 0, C.byref(n)))
    out = np.zeros((n.value, 6), dtype=np.int32)
    check(lib().smc_ce_triangles(out.ctypes.data_as(C.POINTER(C.c_int32)), n.value, None))
    return out


def smc_ce_energy(ctx, ce: dict, snap_ptr, batch, cells_per_axis, e_out_ptr):
    """ce: dict with n_species, pair [3][S][S], triangle [n], species [n][3], J [n]."""
    pair = np.ascontiguousarray(ce["pair"], dtype=np.float64)
    tri = np.ascontiguousarray(ce["triangle"], dtype=np.int32)
    sp = np.ascontiguousarray(ce["species"], dtype=np.uint8)
    J = np.ascontiguousarray(ce["J"], dtype=np.float64)
    s = smc_ce(int(ce["n_species"]), pair.ctypes.data_as(C.POINTER(C.c_double)), len(J),
               tri.ctypes.data_as(C.POINTER(C.c_int32)), sp.ctypes.data_as(C.POINTER(C.c_uint8)),
               J.ctypes.data_as(C.POINTER(C.c_double)))
    check(lib().smc_ce_energy(ctx, C.byref(s), snap_ptr, batch, cells_per_axis, e_out_ptr), ctx)


def smc_n_sites(ctx) -> int:
    n = C.c_int64()
    check(lib().smc_n_sites(ctx, C.byref(n)), ctx)
    return n.value


def smc_n_colours(ctx, replica) -> int:
    n = C.c_int32()
    check(lib().smc_n_colours(ctx, replica, C.byref(n)), ctx)
    return n.value


def smc_destroy(ctx):
    if ctx:
        lib().smc_destroy(ctx)
