"""Loss functionals on the state of a step, with their gradients, for gradient
studies through the adjoint of es_rk3_step (2D RHD and RMHD).

density_squared: L = sum_i w_i rho_i^2 over the interior nodes, with rho from
es_con2prim and dL/dUcurv, dL/dJ by the implicit-function rule at the converged
primitive state, d rho / dU = e_rho^T (dU/dP)^{-1} (U = Ucurv / J, P = (rho, u,
p) with u = W v), the same rule the adjoint applies to con2prim.  dU/dP is
written out from U = (rho W, rho h W u, rho h W^2 - p), h = 1 + Gamma/(Gamma-1)
p/rho, W^2 = 1 + |u|^2.

For 2D RMHD (m = 8, P = (rho, u, p, B)) dU/dP is the Jacobian of U(P) (eq.
RMHDdiv2: D = rho W, m = (Z + |B|^2) v - (v.B) B, E = Z - p - |b|^2/2 + |B|^2,
Z = rho h W^2) by forward-mode differentiation of that map (torch.func).

density_mode_tangents: d Ucurv^0 / d c_m for an initial density rho = 1 + eps
sum_m c_m phi_m at fixed u, p (and B), for the chain rule to the mode
coefficients: dU/drho = (W, W u, W^2) (RHD), (W, W u, W^2, 0) (RMHD).
"""
from __future__ import annotations

import torch


def _interior(c, prim):
    g = 3
    return prim[:, g:-g, g:-g] if c.grid.dim == 2 else prim[:, g:-g, g:-g, g:-g]


def _cons_rmhd(P, G):
    """U(P) of one RMHD state, P = (rho, u_1..3, p, B_1..3)."""
    rho, u, p, B = P[0], P[1:4], P[4], P[5:8]
    W = torch.sqrt(1.0 + (u * u).sum())
    v = u / W
    vB = (v * B).sum()
    BB = (B * B).sum()
    bsq = BB / (W * W) + vB * vB
    Z = (rho + G / (G - 1.0) * p) * W * W
    m = (Z + BB) * v - vB * B
    E = Z - p - 0.5 * bsq + BB
    return torch.cat([(rho * W)[None], m, E[None], B])


def _density_squared_rmhd(ctx, U, J, weight, P):
    G = ctx.scheme_c.gamma
    shape = P.shape[1:]
    Pf = P[:8].reshape(8, -1).T.contiguous()                        # (N, 8)
    A = torch.func.vmap(torch.func.jacfwd(lambda q: _cons_rmhd(q, G)))(Pf)   # (N, 8, 8): dU_r/dP_s
    e0 = torch.zeros(Pf.shape[0], 8, 1, dtype=torch.float64, device=U.device)
    e0[:, 0, 0] = 1.0
    r = torch.linalg.solve(A.transpose(-1, -2), e0)[..., 0]       # d rho / dU, (N, 8)
    rho = P[0]
    L = (weight * rho * rho).sum()
    gU = ((2.0 * weight * rho).reshape(-1, 1) * r).T.reshape((8,) + tuple(shape))
    gUcurv = gU / J
    gJ = -(gU * U).sum(dim=0) / (J * J)
    return L, gUcurv.contiguous(), gJ.contiguous()


def density_squared(ctx, U, J, weight):
    """Returns (L, dL/dUcurv, dL/dJ) for L = sum w rho^2 (2D RHD or RMHD)."""
    if ctx.grid.dim != 2 or ctx.m not in (4, 8):
        raise ValueError("density_squared is written for 2D RHD (m = 4) and 2D RMHD (m = 8)")
    if ctx.m == 8:
        prim = torch.empty((ctx.nprim,) + tuple(ctx.padded_shape()), dtype=torch.float64, device=U.device)
        ctx.con2prim(U, J, prim)
        return _density_squared_rmhd(ctx, U, J, weight, _interior(ctx, prim))
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
    """d Ucurv^0 / d c_m, shape (n_modes, m, *shape), for rho = 1 + eps sum c_m phi_m
    at fixed u, p (and B).  prim0: interior primitive state, (rho, u_1, u_2, p)
    for RHD or (rho, u_1..3, p, B_1..3) for RMHD; phi: (n_modes, *shape)."""
    if ctx.m == 8:
        u = prim0[1:4]
        W = torch.sqrt(1.0 + (u * u).sum(dim=0))
        z = torch.zeros_like(W)
        dU = torch.stack([W, W * u[0], W * u[1], W * u[2], W * W, z, z, z])
        return eps * phi[:, None] * (J * dU)[None]
    u1, u2 = prim0[1], prim0[2]
    W = torch.sqrt(1.0 + u1 * u1 + u2 * u2)
    dU = torch.stack([W, W * u1, W * u2, W * W])                 # (4, *shape)
    return eps * phi[:, None] * (J * dU)[None]
