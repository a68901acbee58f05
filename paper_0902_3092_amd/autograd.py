"""torch.autograd front end of the differentiable PDA solves.

``pda_temperature(ctx, log_rho, kscale, mask, T_D, T_bc)`` returns the PDA
temperature field (one linear solve with the diffusion coefficient frozen at
T_D, eq. T diffusion of Sect. 2.2.1) and is differentiable with respect to the
per-cell log density and extinction scale: the backward pass calls the HIP
adjoint solve (mcrt_pda_adjoint).  ``pda_temperature_nonlinear(ctx, log_rho,
kscale, mask, T_bc)`` is the same for the nonlinear PDA, whose diffusion
coefficient follows the temperature (Sect. 2.2.3): Picard to the fixed point
forward, the adjoint of its Jacobian backward (mcrt_pda_nonlinear,
mcrt_pda_nonlinear_adjoint).  Both directions run in the library.
"""
from __future__ import annotations

import torch

from . import mcrt


class PDAFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, log_rho, kscale, ctx, mask, T_D, T_bc):
        rho = torch.exp(log_rho.detach()).contiguous()
        ks = kscale.detach().contiguous()
        T, _ = ctx.pda_linear(mask, T_D.contiguous(), T_bc.contiguous(), rho=rho, kscale=ks)
        fctx.mcrt_ctx = ctx
        fctx.gen = ctx._lin_gen  # the context keeps only its latest linear solve
        fctx.keep = (rho, ks)    # the saved solve refers to these buffers
        return T

    @staticmethod
    def backward(fctx, grad_T):
        if fctx.mcrt_ctx._lin_gen != fctx.gen:
            raise RuntimeError(
                "pda_temperature: the context has run another PDA solve, batch or hydrostatic "
                "step since this forward; its adjoint would differentiate that instead "
                "(use one context per forward kept for backward)")
        g_logrho, g_ks = fctx.mcrt_ctx.pda_adjoint(grad_T.contiguous())
        return g_logrho, g_ks, None, None, None, None


def pda_temperature(ctx: "mcrt.Context", log_rho, kscale, mask, T_D, T_bc):
    """Differentiable PDA temperature (see module doc).  All tensors float64 on
    the device of the context, [n_cells]; mask uint8."""
    return PDAFunction.apply(log_rho, kscale, ctx, mask, T_D, T_bc)


class PDANonlinearFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, log_rho, kscale, ctx, mask, T_bc):
        rho = torch.exp(log_rho.detach()).contiguous()
        ks = kscale.detach().contiguous()
        T, _ = ctx.pda_nonlinear(mask, T_bc.contiguous(), rho=rho, kscale=ks)
        fctx.mcrt_ctx = ctx
        fctx.gen = ctx._lin_gen
        fctx.keep = (rho, ks)
        return T

    @staticmethod
    def backward(fctx, grad_T):
        if fctx.mcrt_ctx._lin_gen != fctx.gen:
            raise RuntimeError(
                "pda_temperature_nonlinear: the context has run another PDA solve, batch or "
                "hydrostatic step since this forward (use one context per forward kept for "
                "backward)")
        g_logrho, g_ks = fctx.mcrt_ctx.pda_nonlinear_adjoint(grad_T.contiguous())
        return g_logrho, g_ks, None, None, None


def pda_temperature_nonlinear(ctx: "mcrt.Context", log_rho, kscale, mask, T_bc):
    """Differentiable nonlinear PDA temperature (see module doc).  All tensors
    float64 on the device of the context, [n_cells]; mask uint8."""
    return PDANonlinearFunction.apply(log_rho, kscale, ctx, mask, T_bc)
