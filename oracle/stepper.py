"""Oracle time stepping (test infrastructure only).

* CFL time step (eq. cfl): Delta t = CFL / sum_k max_i rho_{k,i} / Delta xi_k, with
  rho_{k,i} the spectral radius of d(F_k)/dU + Phi'(V) dB_k/dU in curvilinear form,
  i.e. L_k max_m |lambda_m(n_k)| / J (mesh-velocity term excluded, as eq. cfl prints it).
* Third-order SSP Runge-Kutta (Proposition 4.2 and the conclusion) in Shu-Osher
  form applied to (U, J), with the stage meshes x^n + c Delta t xdot, c = 0, 1, 1/2,
  and metrics recomputed on each stage mesh.
* One step: con2prim, CFL, mesh redistribution (Section 5), three stages.
"""
from __future__ import annotations

import numpy as np

from . import physics as ph
from . import metrics as mt
from . import residual as rs
from . import dissipation as ds
from . import mesh as msh


def prim_from_cons(grid, scheme, Ucurv, J):
    """U = Ucurv / J, then con2prim; returns full 8-slot primitive P and ok-mask."""
    sel = ph.comps(scheme.phys, grid.dim)
    U = Ucurv / J
    if scheme.phys == ph.RMHD:
        return ph.con2prim_rmhd(U, scheme.gamma)
    return ph.con2prim_rhd(U, scheme.gamma, grid.dim)


def cons_from_prim(grid, scheme, P, J):
    sel = ph.comps(scheme.phys, grid.dim)
    return J * ph.cons(P, scheme.gamma)[sel]


def pad_solution(grid, P, p=3):
    """The primitive state on the box padded by ghost(p) layers (solution rule)."""
    return np.stack([mt.extend(P[c], grid, mt.ghost(p), "solution") for c in range(8)])


def speeds(P, G, phys, dim):
    """Numeric eigenvalues of the (Godunov-Powell modified) x-flux Jacobian at
    states already rotated to the normal frame, shape (N, m)."""
    sel = ph.comps(phys, dim)
    JU = ds._jac(lambda Q: ph.cons(Q, G), P, sel, G)
    JF = ds._jac(lambda Q: ph.flux(Q, G, 0), P, sel, G)
    if phys == ph.RMHD:
        JF = JF.copy()
        JF[:, :, 5] += ph.phi_prime(P, G)[sel].T
    return np.linalg.eigvals(np.linalg.solve(JU, JF)).real


def spectral_radius(grid, scheme, Pin, met, J):
    """rho_{k,i} = L_{k,i} max_m |lambda_m(n_k)| / J_i on the interior, list over k."""
    d = grid.dim
    out = []
    Pflat = Pin.reshape(8, -1)
    for k in range(d):
        a = rs.interior(met[k * (d + 1):(k + 1) * (d + 1)], grid, mt.ghost(scheme.order_p)).reshape(d + 1, -1)
        ax = np.zeros((3, a.shape[1]))
        ax[:d] = a[1:]
        L = np.sqrt(np.sum(ax * ax, axis=0))
        T0 = ds.rotation(ax / L)
        slots = [1, 5] if scheme.phys == ph.RMHD else [1]
        Pr = ds.rotate_full(Pflat, T0, slots)
        lam = speeds(Pr, scheme.gamma, scheme.phys, d)
        out.append((L * np.max(np.abs(lam), axis=1) / J.reshape(-1)).reshape(grid.shape))
    return out


def cfl_dt(grid, scheme, Pin, met, J):
    rho = spectral_radius(grid, scheme, Pin, met, J)
    tot = sum(float(np.max(rho[k])) / grid.dxi[k] for k in range(grid.dim))
    return scheme.cfl / tot


def rk3_step(grid, scheme, mon, Ucurv, J, x, dt=None, details=False, xdot=None, Y_fixed=None):
    """One SSP-RK3 step of the ES adaptive moving-mesh scheme.  ``xdot`` prescribes
    the mesh velocity instead of the adaptive redistribution (the prescribed-motion
    tests of Section 6).  ``Y_fixed``: optional per-stage sign switches (the "Y" list
    of an earlier call with details) used instead of evaluating them.
    Returns dict(U, J, x, xdot, dt, ok)."""
    P0, ok = prim_from_cons(grid, scheme, Ucurv, J)
    if not ok.all():
        return dict(U=Ucurv, J=J, x=x, xdot=np.zeros_like(x), dt=np.nan, ok=ok, dtau=0.0,
                    failed_stage=0)
    met0 = mt.metrics(grid, x, None, scheme.order_p)
    if dt is None:
        dt = cfl_dt(grid, scheme, P0, met0, J)
    if xdot is not None:
        xnew, w, dtau = x + dt * xdot, None, 0.0
    elif mon is not None and mon.enabled:
        xnew, xdot, w, dtau = msh.redistribute(grid, mon, P0, x, dt)
    else:
        xnew, xdot, w, dtau = x.copy(), np.zeros_like(x), None, 0.0
    U0, J0 = Ucurv, J
    P = P0
    coef = (0.0, 1.0, 0.5)
    Us, Js = U0, J0
    Ys = []
    for s in range(3):
        if s > 0:
            P, oks = prim_from_cons(grid, scheme, Us, Js)
            ok = ok & oks
        if not ok.all():
            # an inadmissible state reached con2prim: stop and report (no clipping)
            return dict(U=Ucurv, J=J, x=x, xdot=xdot, dt=dt, ok=ok, dtau=dtau, failed_stage=s)
        xs = x + coef[s] * dt * xdot
        met = mt.metrics(grid, xs, xdot, scheme.order_p)
        L, LJ, info = rs.residual(grid, scheme, pad_solution(grid, P, scheme.order_p), met, details=True,
                                  Y_fixed=None if Y_fixed is None else Y_fixed[s])
        Ys.append({k: info[k]["Y"] for k in info})
        if s == 0:
            Us, Js = U0 + dt * L, J0 + dt * LJ
        elif s == 1:
            Us, Js = 0.75 * U0 + 0.25 * (Us + dt * L), 0.75 * J0 + 0.25 * (Js + dt * LJ)
        else:
            Us, Js = U0 / 3.0 + 2.0 / 3.0 * (Us + dt * L), J0 / 3.0 + 2.0 / 3.0 * (Js + dt * LJ)
    out = dict(U=Us, J=Js, x=xnew, xdot=xdot, dt=dt, ok=ok, dtau=dtau)
    if details:
        out["omega"] = w
        out["Y"] = Ys
    return out


def initial_state(grid, scheme, P, x):
    """J^0 from the mesh and Ucurv^0 = J^0 U(P^0)."""
    J = mt.jacobian(grid, x, scheme.order_p)
    return cons_from_prim(grid, scheme, P, J), J
