"""Loss functionals on the state of a step, with their gradients, for gradient
studies through the adjoint of es_rk3_step (2D RHD).

density_squared: L = sum_i w_i rho_i^2 over the interior nodes, with rho from
es_con2prim and dL/dUcurv, dL/dJ by the implicit-function rule at the converged
primitive state, d rho / dU = e_rho^T (dU/dP)^{-1} (U = Ucurv / J, P = (rho, u,
p) with u = W v), the same rule the adjoint applies to con2prim.  dU/dP is
written out from U = (rho W, rho h W u, rho h W^2 - p), h = 1 + Gamma/(Gamma-1)
p/rho, W^2 = 1 + |u|^2.

density_mode_tangents: d Ucurv^0 / d c_m for an initial density rho = 1 + eps
sum_m c_m phi_m at fixed u and p, for the chain rule to the mode coefficients.
"""
from __future__ import annotations

import torch


def _interior(c, prim):
    g = 3
    return prim[:, g:-g, g:-g] if c.grid.dim == 2 else prim[:, g:-g, g:-g, g:-g]


def density_squared(ctx, U, J, weight):
    """Returns (L, dL/dUcurv, dL/dJ) for L = sum w rho^2 (2D RHD)."""
    if ctx.grid.dim != 2 or ctx.m != 4:
        raise ValueError("density_squared is written for 2D RHD (m = 4)")
    G = ctx.scheme_c.gamma
    prim = torch.empty((ctx.nprim,) + tuple(ctx.padded_shape()), dtype=torch.float64, device=U.device)
    ctx.con2prim(U, J, prim)
    P = _interior(ctx, prim)
    rho, u1, u2, p = P[0], P[1], P[2], P[3]
    L = (weight * rho * rho).sum()
    W = torch.sqrt(1.0 + u1 * u1 + u2 * u2)
    H = rho + G / (G - 1.0) * p                   # rho h
    c = G / (G - 1.0)
    A = torch.zeros(rho.shape + (4, 4), dtype=torch.float64, device=U.device)   # A[r][s] = dU_r/dP_s
    A[..., 0, 0] = W
    A[..., 0, 1] = rho * u1 / W
    A[..., 0, 2] = rho * u2 / W
    for k, uk in ((1, u1), (2, u2)):
        A[..., k, 0] = W * uk
        A[..., k, 1] = H * (uk * u1 / W + (W if k == 1 else 0.0))
        A[..., k, 2] = H * (uk * u2 / W + (W if k == 2 else 0.0))
        A[..., k, 3] = c * W * uk
    A[..., 3, 0] = W * W
    A[..., 3, 1] = 2.0 * H * u1
    A[..., 3, 2] = 2.0 * H * u2
    A[..., 3, 3] = c * W * W - 1.0
    e0 = torch.zeros(rho.shape + (4, 1), dtype=torch.float64, device=U.device)
    e0[..., 0, 0] = 1.0
    r = torch.linalg.solve(A.transpose(-1, -2), e0)[..., 0]       # d rho / dU, (..., 4)
    gU = (2.0 * weight * rho)[..., None] * r                       # dL/dU (U = Ucurv / J)
    gU = gU.permute(2, 0, 1)
    gUcurv = gU / J
    gJ = -(gU * U).sum(dim=0) / (J * J)
    return L, gUcurv.contiguous(), gJ.contiguous()


def density_mode_tangents(ctx, prim0, J, phi, eps):
    """d Ucurv^0 / d c_m, shape (n_modes, 4, *shape), for rho = 1 + eps sum c_m phi_m
    at fixed u, p: dU/drho = (W, W u_1, W u_2, W^2) (2D RHD).  prim0: interior
    primitive state (rho, u_1, u_2, p); phi: (n_modes, *shape)."""
    u1, u2 = prim0[1], prim0[2]
    W = torch.sqrt(1.0 + u1 * u1 + u2 * u2)
    dU = torch.stack([W, W * u1, W * u2, W * W])                 # (4, *shape)
    return eps * phi[:, None] * (J * dU)[None]
