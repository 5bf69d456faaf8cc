"""torch.autograd wrappers over the qx solver and force kernels.

StaggeredSolve.apply(U, b, mass, lat) -> x = A(U)^{-1} b with A = m^2 - D_eo D_oe;
its backward solves the adjoint system (A is Hermitian, so lam = A^{-1} g) and
forms the link gradient with the outer-product kernel.
staggered_action(U, phi, mass, lat) -> S = sum_s phi_s^dag A^{-1} phi_s (one solve;
the backward reuses the G computed in the forward pass).

Gradients follow PyTorch's convention for complex tensors (dL/dRe + i dL/dIm).
"""
from __future__ import annotations

import torch

from . import CG_FP64, CG_MIXED_F32, Gauge, action_backward, cg, force, force_from_fields


def _gauges(lat, U, mixed, recon):
    U = U.detach().contiguous()
    g64 = Gauge(lat, U, "f64", 18)
    glo = Gauge(lat, U, "f32", recon) if mixed else None
    return g64, glo


class StaggeredSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, b, mass, lat, tol=1e-10, mixed=False, recon=18):
        g64, glo = _gauges(lat, U, mixed, recon)
        mode = CG_MIXED_F32 if mixed else CG_FP64
        x, _ = cg(g64, b.detach().contiguous(), float(mass), glo, tol=tol, mode=mode)
        ctx.g = (g64, glo, float(mass), tol, mode)
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        g64, glo, mass, tol, mode = ctx.g
        lam, _ = cg(g64, gx.contiguous(), mass, glo, tol=tol, mode=mode)
        gU = force_from_fields(g64, x, lam) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gU, gb, None, None, None, None, None


class StaggeredAction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, phi, mass, lat, tol=1e-10, mixed=False, recon=18):
        g64, glo = _gauges(lat, U, mixed, recon)
        mode = CG_MIXED_F32 if mixed else CG_FP64
        S, G, x, _ = force(g64, phi.detach().contiguous(), float(mass), glo, tol=tol, mode=mode)
        ctx.lat = lat
        ctx.save_for_backward(G, x)
        return torch.tensor(S, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, gS):
        G, x = ctx.saved_tensors
        # gS * G and 2 gS x (dS/dphi = 2 A^-1 phi) are formed by the library
        gU, gphi = action_backward(ctx.lat, float(gS), G, x, ctx.needs_input_grad[0],
                                   ctx.needs_input_grad[1])
        return gU, gphi, None, None, None, None, None


def staggered_action(U, phi, mass, lat, tol=1e-10, mixed=False, recon=18):
    return StaggeredAction.apply(U, phi, mass, lat, tol, mixed, recon)
