"""CPU-side checks of the C ABI: libes.so builds, loads and exports every entry
point declared in include/es.h; argument validation rejects bad options before
any device work (no GPU needed for these paths)."""
import ctypes
import os
import re

import pytest

from paper_2107_12027_amd import es, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "es.h")


def _ensure_built():
    if not os.path.exists(es.LIB_PATH):
        from paper_2107_12027_amd import build
        build.build()


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:es_status|size_t|const char\*)\s+(es_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("es_metrics", "es_residual", "es_con2prim", "es_mesh_redistribute", "es_rk3_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    lib = ctypes.CDLL(es.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(es.SYMBOLS) == set(declared_symbols())


def _create(grid, scheme, monitor):
    _ensure_built()
    lib = es.load()
    g = es.Grid(grid.dim, (ctypes.c_int * 3)(*grid.n), (ctypes.c_int * 3)(*grid.bc),
                (ctypes.c_double * 3)(*grid.dxi), (ctypes.c_double * 3)(*grid.period))
    s = es.Scheme(scheme.phys, scheme.gamma, scheme.order_p, scheme.dissipation, scheme.mixed,
                  scheme.weno_eps, scheme.cfl)
    m = es.Monitor(monitor.enabled, monitor.sigma, monitor.form, monitor.alpha,
                   monitor.filter_passes, monitor.sweeps, monitor.alpha2)
    h = ctypes.c_void_p()
    return lib.es_create(ctypes.byref(g), ctypes.byref(s), ctypes.byref(m), ctypes.byref(h)), h


@pytest.mark.parametrize("mutate,expect", [
    (lambda g, s, m: setattr(g, "n", (6, 10, 1)), es.ES_EINVAL),          # outflow axis < 7 nodes
    (lambda g, s, m: setattr(g, "dim", 4), es.ES_EINVAL),
    (lambda g, s, m: setattr(s, "gamma", 2.5), es.ES_EINVAL),
    (lambda g, s, m: setattr(s, "cfl", 0.0), es.ES_EINVAL),
    (lambda g, s, m: setattr(s, "dissipation", 2), es.ES_EINVAL),
    (lambda g, s, m: setattr(m, "form", 7), es.ES_EINVAL),
    (lambda g, s, m: setattr(s, "order_p", 5), es.ES_EUNSUPPORTED),
    # p = 4 needs 2 ng + 1 = 9 nodes on outflow axes (four ghost layers)
    (lambda g, s, m: (setattr(s, "order_p", 4), setattr(g, "n", (8, 10, 1))), es.ES_EINVAL),
    (lambda g, s, m: (setattr(s, "order_p", 1), setattr(s, "phys", 1)), es.ES_EUNSUPPORTED),
    (lambda g, s, m: (setattr(m, "enabled", 1), setattr(m, "form", 2), setattr(m, "alpha2", -1.0)),
     es.ES_EINVAL),
    (lambda g, s, m: setattr(s, "phys", 2), es.ES_EINVAL),
])
def test_create_rejects_bad_options_before_device_work(mutate, expect):
    w = wl.quadrant_riemann(n=10)
    mutate(w.grid, w.scheme, w.monitor)
    st, h = _create(w.grid, w.scheme, w.monitor)
    assert st == expect
    assert not h.value


def test_status_strings():
    lib = es.load() if os.path.exists(es.LIB_PATH) else None
    if lib is None:
        _ensure_built()
        lib = es.load()
    for code in range(8):
        assert lib.es_status_string(code)
    assert lib.es_status_string(99) == b"unknown status"
