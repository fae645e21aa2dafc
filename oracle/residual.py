"""Oracle semi-discrete residual (test infrastructure only).

The 2p-th order scheme of Section 3.2 with the ES flux of Section 4:
  dU_i/dt = - sum_k 1/dxi_k (F^_{i,k,+1/2} - F^_{i,k,-1/2})
            - Phi'(V_i)^T sum_k 1/dxi_k (B~_{i,k,+1/2} - B~_{i,k,-1/2})   (eq. RMHDSemiU_O2p_ES)
  dJ_i/dt = - sum_k 1/dxi_k ((J xi_t)~_{i,k,+1/2} - (J xi_t)~_{i,k,-1/2})  (eq. RMHDSemiJ_O2p_ES)
with the interface fluxes built literally as in Proposition 4.1:
  F~^{2p}_{i+1/2} = sum_{n=1}^{p} alpha_{p,n} sum_{s=0}^{n-1} F~(i-s, i-s+n)     (eq. ECFlux_O2p)
and likewise for B~ (eq. BFlux_O2p) and the VCL flux (eq. MetricsFlux_O2p).
Inputs: full 8-slot primitive states and metrics on the ghost-padded box.
"""
from __future__ import annotations

import numpy as np

from . import physics as ph
from . import ecflux as ec
from . import dissipation as ds
from .metrics import alpha, crop, ghost


def _line_view(arr, grid, k, lead, ng=3):
    """Crop every axis except k to the interior (``ng`` ghost layers); ``lead``
    leading non-spatial axes."""
    out = arr
    nd = arr.ndim - lead
    for kk in range(grid.dim):
        if kk != k:
            out = crop(out, lead + nd - 1 - kk, ng)
    return out


def _take(a, idx, ax):
    return np.take(a, idx, axis=ax)


def residual(grid, scheme, Ppad, met, details=False, Y_fixed=None, eig_fixed=None):
    """Returns (dU (m, *shape), dJ (*shape)) on the interior nodes, optionally with
    per-direction face fluxes and sign switches.  Y_fixed: optional {direction:
    Y (m, faces)} from an earlier call with details, used instead of evaluating
    the switch.  eig_fixed: optional {direction: (R, lhat)} from an earlier call
    with details, used instead of the face eigen-structure (both for difference
    quotients with the decisions and the eigen-structure held)."""
    d = grid.dim
    G = scheme.gamma
    phys = scheme.phys
    p = scheme.order_p
    ng = ghost(p)
    al = alpha(p)
    sel = ph.comps(phys, d)
    shape = grid.shape
    dU = np.zeros((8,) + shape)
    dJ = np.zeros(shape)
    src = np.zeros(shape)
    info = {}
    for k in range(d):
        ax_sp = d - 1 - k                     # spatial axis of direction k
        Pk = _line_view(Ppad, grid, k, 1, ng)     # (8, ..., n_k + 2 ng, ...)
        ak = _line_view(met[k * (d + 1):(k + 1) * (d + 1)], grid, k, 1, ng)
        nk = grid.n[k]
        faces = np.arange(ng - 1, ng + nk)    # face I+1/2 between padded nodes I, I+1
        Ff = 0.0
        Bf = 0.0
        Jf = 0.0
        for n in range(1, p + 1):
            for s in range(n):
                li = faces - s
                ri = faces - s + n
                Pl, Pr = _take(Pk, li, 1 + ax_sp), _take(Pk, ri, 1 + ax_sp)
                aL, aR = _take(ak, li, 1 + ax_sp), _take(ak, ri, 1 + ax_sp)
                Ff = Ff + al[n - 1] * ec.curvilinear_pair(Pl, Pr, aL, aR, G, phys, d)
                if phys == ph.RMHD:
                    Bf = Bf + al[n - 1] * ec.curvilinear_pair_B(Pl, Pr, aL, aR, d)
                Jf = Jf + al[n - 1] * ec.curvilinear_pair_Jt(aL, aR)
        if scheme.dissipation:
            fshape = Ff.shape[1:]
            # WENO-(2p-1) on the 2p nodes i-p+1..i+p of each face
            Pst = np.stack([_take(Pk, faces + j, 1 + ax_sp) for j in range(1 - p, p + 1)])
            ast = np.stack([_take(ak, faces + j, 1 + ax_sp) for j in range(0, 2)])
            Pst = Pst.reshape(2 * p, 8, -1)
            ast = ast.reshape(2, d + 1, -1)
            dd, dinfo = ds.face_dissipation(Pst, ast, G, phys, d, scheme.weno_eps, details=True,
                                            Y_fixed=None if Y_fixed is None else Y_fixed[k],
                                            eig_fixed=None if eig_fixed is None else eig_fixed[k])
            Ff = Ff - 0.5 * dd.reshape((8,) + fshape)
            Yk = dinfo["Y"]
            eigk = (dinfo["R"], dinfo["lhat"])
            lamk = dinfo["lam"]
            groupk = dict(ds.last_group_decisions) if phys == ph.RMHD else None
        hi = np.arange(1, nk + 1)
        lo = np.arange(0, nk)
        dxi = grid.dxi[k]
        dU -= (_take(Ff, hi, 1 + ax_sp) - _take(Ff, lo, 1 + ax_sp)) / dxi
        dJ -= (_take(Jf, hi, ax_sp) - _take(Jf, lo, ax_sp)) / dxi
        if phys == ph.RMHD:
            src += (_take(Bf, hi, ax_sp) - _take(Bf, lo, ax_sp)) / dxi
        if details:
            info[k] = dict(F=Ff, J=Jf, B=Bf, Y=Yk if scheme.dissipation else None,
                           eig=eigk if scheme.dissipation else None,
                           lam=lamk if scheme.dissipation else None,
                           groups=groupk if scheme.dissipation else None)
    if phys == ph.RMHD:
        Pin = interior(Ppad, grid, ng)
        dU -= ph.phi_prime(Pin, G) * src
    if details:
        return dU[sel], dJ, info
    return dU[sel], dJ


def interior(Ppad, grid, ng=3):
    """The interior nodes of a field on the box padded by ``ng`` ghost layers."""
    out = Ppad
    for k in range(grid.dim):
        out = crop(out, out.ndim - 1 - k, ng)
    return out


def entropy_production(grid, scheme, Pin, dU, dJ):
    """sum_i (V_i . dU_i/dt - phi_i dJ_i/dt) = d/dt sum_i J_i eta_i (chain rule with
    phi = V.U - eta); zero for the EC scheme on periodic meshes (Theorem 4.1) and
    non-positive for the ES scheme (Theorem 5.1)."""
    sel = ph.comps(scheme.phys, grid.dim)
    V = ph.entropy_vars(Pin, scheme.gamma)[sel]
    phi, _, _ = ph.potentials(Pin, scheme.gamma)
    return float(np.sum(np.sum(V * dU, axis=0) - phi * dJ))
