"""The allocation-free CFL step (es_cfl_noalloc: no context, block maxima in a
static device array) against es_cfl on the same inputs, through the C ABI: two
calls in a row, the second on a smaller grid, bit for bit (maxima are exact in
any order and both run the same kernels); grids beyond the static scratch are
refused before anything is enqueued."""
import ctypes
import os

import numpy as np
import pytest

from gpu_util import Case, empty, host
from oracle import physics as ph
from paper_2107_12027_amd import es, workloads as wl


def _cfl_both(case):
    from gpu_util import dev
    c = case.ctx
    U, J = case.gpu_state()
    prim = empty(c.nprim, *c.padded_shape())
    met = empty(c.nmet, *c.padded_shape())
    c.con2prim(U, J, prim)
    c.metrics(dev(case.x), None, met)
    dt_ref, dt_na = empty(1), empty(1)
    c.cfl(prim, met, J, dt_ref)
    c.cfl_noalloc(prim, met, J, dt_na)
    assert c.status()[0] == es.ES_OK
    return float(host(dt_ref)[0]), float(host(dt_na)[0])


@pytest.mark.gpu
@pytest.mark.parametrize("phys,first,second", [
    (ph.RHD, (3, (40, 36, 33), (0, 1, 1)), (2, (70, 9, 1), (1, 0, 0))),
    (ph.RMHD, (2, (300, 260, 1), (1, 1, 0)), (2, (33, 21, 1), (0, 0, 0))),
])
def test_cfl_noalloc_matches_cfl_twice(phys, first, second):
    for dim, n, bc in (first, second):
        case = Case(dim, n, bc, phys=phys, seed=17 + dim, vmax=0.9)
        ref, na = _cfl_both(case)
        assert np.isfinite(ref) and ref > 0
        assert na == ref, (n, na, ref)


def test_cfl_noalloc_refuses_grids_beyond_the_scratch():
    # checked on the host before any device work (no GPU needed)
    if not os.path.exists(es.LIB_PATH):
        from paper_2107_12027_amd import build
        build.build()
    lib = es.load()
    g = wl.make_grid(3, (512, 512, 512), (0, 0, 0))
    gc = es.Grid(3, (ctypes.c_int * 3)(*g.n), (ctypes.c_int * 3)(*g.bc), (ctypes.c_double * 3)(*g.dxi),
                 (ctypes.c_double * 3)(*g.period))
    sc = es.Scheme(0, 5.0 / 3.0, 3, 1, 0, 1e-6, 0.3)
    assert lib.es_cfl_static_blocks(ctypes.byref(gc)) == 8 * 128 * 512
    fake = ctypes.c_void_p(256)      # never dereferenced: the size check comes first
    st = lib.es_cfl_noalloc(ctypes.byref(gc), ctypes.byref(sc), fake, fake, fake, fake, None)
    assert st == es.ES_ETOOLARGE
    assert lib.es_status_string(st).decode().startswith("grid exceeds")
    g2 = wl.make_grid(2, (4096, 4 * 32768, 1), (0, 0, 0))
    gc2 = es.Grid(2, (ctypes.c_int * 3)(*g2.n), (ctypes.c_int * 3)(*g2.bc), (ctypes.c_double * 3)(*g2.dxi),
                  (ctypes.c_double * 3)(*g2.period))
    assert lib.es_cfl_static_blocks(ctypes.byref(gc2)) == 64 * 32768
    assert lib.es_cfl_noalloc(ctypes.byref(gc2), ctypes.byref(sc), fake, fake, fake, fake, None) == es.ES_ETOOLARGE
