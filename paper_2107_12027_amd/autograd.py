"""torch.autograd.Function around one SSP-RK3 step of libes.so.

Forward: es_rk3_step_save, which advances (Ucurv, J, x) and writes the step's
checkpoint (stage states, mesh, mesh velocity, time step) into a device tensor
kept for the backward pass.  Backward: es_rk3_step_vjp, the hand-written
adjoint of the step (transposed residual stencils, the implicit-function rule
for con2prim, the Runge-Kutta stages in reverse).  The mesh trajectory, the
time step and every branch decision of the scheme are held at their forward
values, so for a static mesh and a fixed time step the gradient is exact.
Argument marshalling only; the arithmetic runs in the library's kernels.
"""
from __future__ import annotations

import torch


class RK3Step(torch.autograd.Function):
    """(Ucurv, J) -> (Ucurv', J') for one step on the context's mesh x.

    Inputs: Ucurv (m, *shape), J (*shape), the es.Context, the mesh x (d, *shape)
    and optionally a device time step fixed_dt (1,) used instead of the CFL step.
    Outputs: Ucurv', J', the new mesh x' and the time step dt (the last two are
    not differentiable)."""

    @staticmethod
    def forward(fctx, U, J, es_ctx, x, fixed_dt=None):
        Un = U.detach().clone().contiguous()
        Jn = J.detach().clone().contiguous()
        xn = x.detach().clone().contiguous()
        xdot = torch.empty_like(xn)
        dt = torch.empty(1, dtype=torch.float64, device=U.device)
        ckpt = torch.empty(es_ctx.ckpt_doubles(), dtype=torch.float64, device=U.device)
        es_ctx.rk3_step_save(Un, Jn, xn, xdot, dt, ckpt, fixed_dt)
        fctx.save_for_backward(ckpt)
        fctx.es_ctx = es_ctx
        fctx.mark_non_differentiable(xn, dt)
        return Un, Jn, xn, dt

    @staticmethod
    def backward(fctx, gU, gJ, gx, gdt):
        (ckpt,) = fctx.saved_tensors
        es_ctx = fctx.es_ctx
        shape = tuple(es_ctx.shape())
        dev = ckpt.device
        lamU = gU.contiguous() if gU is not None else torch.zeros((es_ctx.m,) + shape, dtype=torch.float64, device=dev)
        lamJ = gJ.contiguous() if gJ is not None else torch.zeros(shape, dtype=torch.float64, device=dev)
        outU = torch.empty_like(lamU)
        outJ = torch.empty_like(lamJ)
        es_ctx.rk3_step_vjp(ckpt, lamU, lamJ, outU, outJ)
        return outU, outJ, None, None, None


def rk3_step(U, J, es_ctx, x, fixed_dt=None):
    """Differentiable step: returns (Ucurv', J', x', dt)."""
    return RK3Step.apply(U, J, es_ctx, x, fixed_dt)
