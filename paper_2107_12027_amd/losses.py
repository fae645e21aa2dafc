"""Loss functionals on the state of a step, for gradient studies through the
adjoint of es_rk3_step (2D and 3D, RHD and RMHD).

Every derivative of the method's maps runs in the library: the density comes
from es_con2prim and its cotangent is pulled back to (Ucurv, J) by
es_con2prim_vjp (the implicit-function rule at the converged primitive state);
the chain to parameters of the initial primitive state goes through
es_prim2con_vjp.  What is left here is the loss itself (a weighted sum of
squares) and the projection of a primitive cotangent onto parameter modes.

density_squared: L = sum_i w_i rho_i^2 over the interior nodes; returns L and
dL/dUcurv, dL/dJ.

density_mode_gradient: for an initial density rho = rho_0 + eps sum_m c_m phi_m
at fixed u, p (and B) and a cotangent gU0 of Ucurv^0 = J^0 U(P^0), the gradient
dL/dc_m = eps sum_i phi_m,i (J^0 (dU/dP)^T gU0)_rho,i.
"""
from __future__ import annotations

import torch


def _interior(ctx, prim):
    g = ctx.ng
    return prim[:, g:-g, g:-g] if ctx.grid.dim == 2 else prim[:, g:-g, g:-g, g:-g]


def density_squared(ctx, U, J, weight):
    """Returns (L, dL/dUcurv, dL/dJ) for L = sum w rho^2."""
    prim = torch.empty((ctx.nprim,) + tuple(ctx.padded_shape()), dtype=torch.float64, device=U.device)
    ctx.con2prim(U, J, prim)
    rho = _interior(ctx, prim)[0]
    L = (weight * rho * rho).sum()
    gprim = torch.zeros((ctx.m,) + tuple(ctx.shape()), dtype=torch.float64, device=U.device)
    gprim[0] = 2.0 * weight * rho
    gU = torch.empty_like(U)
    gJ = torch.empty_like(J)
    ctx.con2prim_vjp(U, J, gprim, gU, gJ)
    return L, gU, gJ


def density_mode_gradient(ctx, prim0, J0, gU0, phi, eps):
    """dL/dc_m, shape (n_modes,), from the cotangent gU0 of Ucurv^0 = J^0 U(prim0).
    prim0: interior primitive state in the es_prim2con layout (m comps); phi:
    (n_modes, *shape)."""
    gprim = torch.empty((ctx.m,) + tuple(ctx.shape()), dtype=torch.float64, device=gU0.device)
    ctx.prim2con_vjp(prim0, J0, gU0, gprim)
    dims = tuple(range(1, phi.dim()))
    return eps * (phi * gprim[0][None]).sum(dim=dims)
