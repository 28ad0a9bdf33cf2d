"""Host-only checks of the C ABI: the library loads, exports what include/smc.h declares,
and rejects invalid configurations before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smc_[a-z0-9_]+)\s*\(", text)))


def _lib():
    from paper_2604_08250_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libsmc.so not built")
    return L


def test_library_exports_every_declared_symbol():
    L = _lib()
    names = _declared("smc.h")
    assert "smc_init" in names and "smc_sweep" in names and "smc_energy" in names
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), n
    # the Python binding marshals exactly the declared entry points
    assert set(names) == set(L.EXPORTS)


def _cfg(L, cells=((8, 8, 8),), temps=(1000.0,), n_species=4, feature=0, hidden=64, precision=0):
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int32))
    temps = np.ascontiguousarray(np.asarray(temps, dtype=np.float64))
    cfg = L.smc_config(len(temps), cells.ctypes.data_as(C.POINTER(C.c_int32)),
                       temps.ctypes.data_as(C.POINTER(C.c_double)), n_species, feature, hidden,
                       precision, 0, -1.0)
    return cfg, (cells, temps)


@pytest.mark.parametrize("kw,code", [
    (dict(cells=((3, 8, 8),)), -1),            # edge below 4
    (dict(n_species=1), -1),
    (dict(n_species=6), -1),
    (dict(feature=7), -1),
    (dict(hidden=96), -2),
    (dict(precision=9), -1),
    (dict(temps=(-5.0,)), -1),
    (dict(temps=(float("nan"),)), -1),
])
def test_invalid_configurations_are_rejected(kw, code):
    L = _lib()
    cfg, keep = _cfg(L, **kw)
    ctx = C.c_void_p()
    dummy = C.c_void_p(16)  # never dereferenced: validation happens first
    rc = L.lib().smc_init(C.byref(cfg), dummy, dummy, dummy, None, C.byref(ctx))
    assert rc == code
    assert not ctx.value


def test_null_arguments():
    L = _lib()
    lib = L.lib()
    assert lib.smc_init(None, None, None, None, None, None) == -1
    assert lib.smc_sweep(None, 1, None) == -1
    assert lib.smc_energy(None, None, None) == -1
    assert lib.smc_set_temperatures(None, None) == -1
    assert lib.smc_lattice_shells(7, None, None, 0) == -1
    assert lib.smc_warren_cowley(None, 0, None) == -1
    assert lib.smc_set_strategy(None, 1) == -1
    assert lib.smc_get_strategy(None, None) == -1
    assert lib.smc_use_graph(None, 1) == -1
    assert lib.smc_set_variant(None, 0) == -1
    assert lib.smc_get_variant(None, None) == -1
    assert lib.smc_autotune(None, None, None, None) == -1
    assert lib.smc_status_string(-3) == b"device error"
    lib.smc_destroy(None)


def test_library_triangle_shapes_equal_oracle():
    """The CE triangle-shape list is index data shared by contract: bit-exact equality."""
    L = _lib()
    import oracle
    assert np.array_equal(L.smc_ce_triangles(), oracle.ce_triangles())


def test_fit_entry_points_reject_null_context():
    L = _lib()
    lib = L.lib()
    assert lib.smc_energy_fwd(None, None, 1, 4, None, None) == -1
    assert lib.smc_energy_bwd(None, None, 1, 4, None, None, None) == -1
    assert lib.smc_fit_step(None, None, 1, 4, None, None, None, None, 1e-3, 1, None) == -1
    assert lib.smc_ce_energy(None, None, None, 1, 4, None) == -1


def test_lattice_shells_equal_the_oracles():
    """The library's neighbour slot tables (BCC and FCC) equal the oracle's, slot for slot."""
    import numpy as np
    import oracle
    from oracle import fcc
    import paper_2604_08250_amd as smc
    off, sh = smc.smc_lattice_shells(smc.SMC_LATTICE_BCC)
    o, s = oracle.shell_table()
    assert np.array_equal(off, o) and np.array_equal(sh, s)
    off, sh = smc.smc_lattice_shells(smc.SMC_LATTICE_FCC)
    o, s = fcc.shell_table()
    assert np.array_equal(off, o) and np.array_equal(sh, s)
