"""ctypes binding of libes.so (include/es.h).

Argument marshalling only: every computation runs in the HIP kernels of the
library.  Arrays are torch tensors on the GPU (float64, contiguous); the binding
passes their data pointers and the current HIP stream.  If the library is not
built, or is loaded on a machine without a GPU, the calls fail loudly: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libes.so")

ES_OK, ES_EINVAL, ES_EADMISSIBLE, ES_ENOCONV, ES_EMESH, ES_EHIP, ES_EUNSUPPORTED, ES_ETOOLARGE = range(8)
SYMBOLS = ("es_create", "es_destroy", "es_nvars", "es_nprim", "es_nmet", "es_nodes",
           "es_padded_nodes", "es_ghost_layers", "es_prim2con", "es_metrics", "es_con2prim", "es_residual",
           "es_cfl", "es_mesh_redistribute", "es_rk3_step", "es_rk3_step_moving", "es_set_graph",
           "es_diagnostics", "es_ctx_status", "es_status_string", "es_ckpt_doubles", "es_rk3_step_save",
           "es_rk3_step_vjp", "es_residual_vjp", "es_con2prim_vjp", "es_prim2con_vjp",
           "es_cfl_static_blocks", "es_cfl_noalloc")


class EsError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__("%s failed: %s (status %d)" % (where, msg, status))
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("bc", ctypes.c_int * 3),
                ("dxi", ctypes.c_double * 3), ("period", ctypes.c_double * 3)]


class Scheme(ctypes.Structure):
    _fields_ = [("phys", ctypes.c_int), ("gamma", ctypes.c_double), ("order_p", ctypes.c_int),
                ("dissipation", ctypes.c_int), ("mixed", ctypes.c_int),
                ("weno_eps", ctypes.c_double), ("cfl", ctypes.c_double)]


class Monitor(ctypes.Structure):
    _fields_ = [("enabled", ctypes.c_int), ("sigma", ctypes.c_int), ("form", ctypes.c_int),
                ("alpha", ctypes.c_double), ("filter_passes", ctypes.c_int),
                ("sweeps", ctypes.c_int), ("alpha2", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libes.so (built by paper_2107_12027_amd.build); raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libes.so is not built: run `python -m paper_2107_12027_amd.build` "
                           "(no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    st = ctypes.c_int
    lib.es_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Scheme), ctypes.POINTER(Monitor),
                              ctypes.POINTER(vp)]
    lib.es_create.restype = st
    lib.es_destroy.argtypes = [vp]
    lib.es_destroy.restype = st
    for name in ("es_nvars", "es_nprim", "es_nmet", "es_nodes", "es_padded_nodes", "es_ghost_layers"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = ctypes.c_size_t
    lib.es_prim2con.argtypes = [vp, vp, vp, vp, vp]
    lib.es_metrics.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.es_con2prim.argtypes = [vp, vp, vp, vp, vp]
    lib.es_residual.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.es_cfl.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.es_mesh_redistribute.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.es_rk3_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.es_rk3_step_moving.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.es_diagnostics.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.es_set_graph.argtypes = [vp, ctypes.c_int]
    lib.es_ctx_status.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_longlong),
                                  ctypes.POINTER(ctypes.c_longlong)]
    lib.es_ckpt_doubles.argtypes = [vp]
    lib.es_ckpt_doubles.restype = ctypes.c_size_t
    lib.es_rk3_step_save.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.es_rk3_step_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.es_residual_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.es_con2prim_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.es_prim2con_vjp.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.es_cfl_static_blocks.argtypes = [ctypes.POINTER(Grid)]
    lib.es_cfl_static_blocks.restype = ctypes.c_size_t
    lib.es_cfl_noalloc.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Scheme), vp, vp, vp, vp, vp]
    for name in ("es_prim2con", "es_metrics", "es_con2prim", "es_residual", "es_cfl",
                 "es_mesh_redistribute", "es_rk3_step", "es_rk3_step_moving", "es_set_graph",
                 "es_diagnostics", "es_ctx_status", "es_rk3_step_save", "es_rk3_step_vjp", "es_residual_vjp",
                 "es_con2prim_vjp", "es_prim2con_vjp", "es_cfl_noalloc"):
        getattr(lib, name).restype = st
    lib.es_status_string.argtypes = [st]
    lib.es_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != ES_OK:
        msg = _lib.es_status_string(status).decode()
        raise EsError(status, where, msg)


def _ptr(t, numel: Optional[int] = None, name: str = "array") -> Optional[int]:
    """Device pointer of a contiguous float64 GPU tensor; with ``numel`` the tensor
    must hold exactly that many elements (the library reads and writes that many
    through the pointer)."""
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("%s: expected a contiguous float64 GPU tensor" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s: expected %d elements, got %d" % (name, numel, t.numel()))
    return t.data_ptr()


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Context:
    """An es_ctx: grid, scheme, monitor and the device workspace of the library."""

    def __init__(self, grid, scheme, monitor):
        lib = load()
        self.grid_c = Grid(grid.dim, (ctypes.c_int * 3)(*grid.n), (ctypes.c_int * 3)(*grid.bc),
                           (ctypes.c_double * 3)(*grid.dxi), (ctypes.c_double * 3)(*grid.period))
        self.scheme_c = Scheme(scheme.phys, scheme.gamma, scheme.order_p, scheme.dissipation,
                               scheme.mixed, scheme.weno_eps, scheme.cfl)
        self.monitor_c = Monitor(monitor.enabled, monitor.sigma, monitor.form, monitor.alpha,
                                 monitor.filter_passes, monitor.sweeps, monitor.alpha2)
        h = ctypes.c_void_p()
        _check(lib.es_create(ctypes.byref(self.grid_c), ctypes.byref(self.scheme_c),
                             ctypes.byref(self.monitor_c), ctypes.byref(h)), "es_create")
        self.h = h
        self.grid = grid
        self.m = lib.es_nvars(h)
        self.nprim = lib.es_nprim(h)
        self.nmet = lib.es_nmet(h)
        self.nodes = lib.es_nodes(h)
        self.pnodes = lib.es_padded_nodes(h)
        self.ng = lib.es_ghost_layers(h)
        self.dim = grid.dim

    def close(self):
        if self.h:
            _lib.es_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes -------------------------------------------------------------
    def shape(self):
        return tuple(self.grid.shape)

    def padded_shape(self):
        return tuple(s + 2 * self.ng for s in self.grid.shape)

    # sizes of the documented layouts ---------------------------------------
    def _int(self, comps=1):
        return comps * self.nodes

    def _pad(self, comps):
        return comps * self.pnodes

    # entry points ---------------------------------------------------------
    def prim2con(self, prim, J, U, stream=None):
        _check(_lib.es_prim2con(self.h, _ptr(prim, self._int(self.m), "prim"), _ptr(J, self._int(), "J"),
                                _ptr(U, self._int(self.m), "U"), _stream(stream)), "es_prim2con")

    def metrics(self, x, xdot, met, J0=None, stream=None):
        d = self.dim
        _check(_lib.es_metrics(self.h, _ptr(x, self._int(d), "x"), _ptr(xdot, self._int(d), "xdot"),
                               _ptr(met, self._pad(self.nmet), "met"), _ptr(J0, self._int(), "J0"),
                               _stream(stream)), "es_metrics")

    def con2prim(self, U, J, prim, stream=None):
        _check(_lib.es_con2prim(self.h, _ptr(U, self._int(self.m), "U"), _ptr(J, self._int(), "J"),
                                _ptr(prim, self._pad(self.nprim), "prim"), _stream(stream)), "es_con2prim")

    def residual(self, prim, met, dU, dJ, stream=None):
        _check(_lib.es_residual(self.h, _ptr(prim, self._pad(self.nprim), "prim"),
                                _ptr(met, self._pad(self.nmet), "met"), _ptr(dU, self._int(self.m), "dU"),
                                _ptr(dJ, self._int(), "dJ"), _stream(stream)), "es_residual")

    def cfl(self, prim, met, J, dt, stream=None):
        _check(_lib.es_cfl(self.h, _ptr(prim, self._pad(self.nprim), "prim"), _ptr(met, self._pad(self.nmet), "met"),
                           _ptr(J, self._int(), "J"), _ptr(dt, 1, "dt"), _stream(stream)), "es_cfl")

    def mesh_redistribute(self, prim, x, dt, x_new, xdot, dtau=None, stream=None):
        d = self.dim
        _check(_lib.es_mesh_redistribute(self.h, _ptr(prim, self._pad(self.nprim), "prim"),
                                         _ptr(x, self._int(d), "x"), _ptr(dt, 1, "dt"),
                                         _ptr(x_new, self._int(d), "x_new"), _ptr(xdot, self._int(d), "xdot"),
                                         _ptr(dtau, 1, "dtau"), _stream(stream)), "es_mesh_redistribute")

    def _step_ptrs(self, U, J, x, xdot, dt, fixed_dt):
        d = self.dim
        return (_ptr(U, self._int(self.m), "U"), _ptr(J, self._int(), "J"), _ptr(x, self._int(d), "x"),
                _ptr(xdot, self._int(d), "xdot"), _ptr(dt, 1, "dt"), _ptr(fixed_dt, 1, "fixed_dt"))

    def rk3_step(self, U, J, x, xdot, dt, fixed_dt=None, stream=None):
        _check(_lib.es_rk3_step(self.h, *self._step_ptrs(U, J, x, xdot, dt, fixed_dt), _stream(stream)),
               "es_rk3_step")

    def rk3_step_moving(self, U, J, x, xdot, dt, fixed_dt=None, stream=None):
        """One step with the caller's mesh velocity ``xdot`` held over the step."""
        _check(_lib.es_rk3_step_moving(self.h, *self._step_ptrs(U, J, x, xdot, dt, fixed_dt), _stream(stream)),
               "es_rk3_step_moving")

    def ckpt_doubles(self) -> int:
        return _lib.es_ckpt_doubles(self.h)

    def rk3_step_save(self, U, J, x, xdot, dt, ckpt, fixed_dt=None, stream=None):
        _check(_lib.es_rk3_step_save(self.h, *self._step_ptrs(U, J, x, xdot, dt, fixed_dt),
                                     _ptr(ckpt, self.ckpt_doubles(), "ckpt"), _stream(stream)), "es_rk3_step_save")

    def rk3_step_vjp(self, ckpt, lamU, lamJ, gU, gJ, stream=None):
        nU, nJ = self._int(self.m), self._int()
        _check(_lib.es_rk3_step_vjp(self.h, _ptr(ckpt, self.ckpt_doubles(), "ckpt"), _ptr(lamU, nU, "lamU"),
                                    _ptr(lamJ, nJ, "lamJ"), _ptr(gU, nU, "gU"), _ptr(gJ, nJ, "gJ"),
                                    _stream(stream)), "es_rk3_step_vjp")

    def residual_vjp(self, U, J, met, lamU, gU, gJ, stream=None):
        nU, nJ = self._int(self.m), self._int()
        _check(_lib.es_residual_vjp(self.h, _ptr(U, nU, "U"), _ptr(J, nJ, "J"), _ptr(met, self._pad(self.nmet), "met"),
                                    _ptr(lamU, nU, "lamU"), _ptr(gU, nU, "gU"), _ptr(gJ, nJ, "gJ"),
                                    _stream(stream)), "es_residual_vjp")

    def con2prim_vjp(self, U, J, gprim, gU, gJ, stream=None):
        """gU, gJ = cotangents of (Ucurv, J) from the cotangent gprim of the interior
        primitive state recovered by con2prim (implicit-function rule)."""
        nU, nJ = self._int(self.m), self._int()
        _check(_lib.es_con2prim_vjp(self.h, _ptr(U, nU, "U"), _ptr(J, nJ, "J"), _ptr(gprim, nU, "gprim"),
                                    _ptr(gU, nU, "gU"), _ptr(gJ, nJ, "gJ"), _stream(stream)), "es_con2prim_vjp")

    def prim2con_vjp(self, prim, J, gU, gprim, gJ=None, stream=None):
        """gprim (and gJ) = cotangents of (prim, J) of Ucurv = J U(prim) from gU."""
        nU, nJ = self._int(self.m), self._int()
        _check(_lib.es_prim2con_vjp(self.h, _ptr(prim, nU, "prim"), _ptr(J, nJ, "J"), _ptr(gU, nU, "gU"),
                                    _ptr(gprim, nU, "gprim"), _ptr(gJ, nJ, "gJ"), _stream(stream)),
               "es_prim2con_vjp")

    def cfl_noalloc(self, prim, met, J, dt, stream=None):
        """es_cfl_noalloc on this context's grid and scheme (the library call takes no
        context and allocates nothing: its block maxima live in a static device array)."""
        _check(_lib.es_cfl_noalloc(ctypes.byref(self.grid_c), ctypes.byref(self.scheme_c),
                                   _ptr(prim, self._pad(self.nprim), "prim"), _ptr(met, self._pad(self.nmet), "met"),
                                   _ptr(J, self._int(), "J"), _ptr(dt, 1, "dt"), _stream(stream)), "es_cfl_noalloc")

    def set_graph(self, enable: bool):
        _check(_lib.es_set_graph(self.h, int(bool(enable))), "es_set_graph")

    def diagnostics(self, prim, U, J, dU, dJ, out, stream=None):
        nU, nJ = self._int(self.m), self._int()
        _check(_lib.es_diagnostics(self.h, _ptr(prim, self._pad(self.nprim), "prim"), _ptr(U, nU, "U"),
                                   _ptr(J, nJ, "J"), _ptr(dU, nU, "dU"), _ptr(dJ, nJ, "dJ"),
                                   _ptr(out, 3 + self.m, "out"), _stream(stream)), "es_diagnostics")

    def status(self, stream=None):
        """Synchronise and return (status, n_fail, first_fail) of the failures recorded
        by con2prim (ES_EMESH: a non-positive Jacobian; ES_EADMISSIBLE; ES_ENOCONV)."""
        nf = ctypes.c_longlong()
        ff = ctypes.c_longlong()
        st = _lib.es_ctx_status(self.h, _stream(stream), ctypes.byref(nf), ctypes.byref(ff))
        if st not in (ES_OK, ES_EADMISSIBLE, ES_ENOCONV, ES_EMESH):
            _check(st, "es_ctx_status")
        return st, nf.value, ff.value


def exported_symbols(path: str = LIB_PATH):
    """Names of the C-ABI entry points exported by libes.so (ctypes lookup only,
    nothing is executed)."""
    lib = ctypes.CDLL(path)
    return [s for s in SYMBOLS if hasattr(lib, s)]
