"""torch.autograd binding of the amplitude cost with the hand-written adjoint.

``amplitude_loss(ctx, obj, probe, pos, meas)`` returns F(V) (Eq. 1) as a
float64 scalar tensor.  Its forward runs the loss-only fused kernel and keeps
nothing but the inputs; its backward calls the fused loss+gradient kernel,
which runs the multislice forward again for every position, keeps the
incident waves of that position only for the duration of its own adjoint
sweep, and scatter-adds dF/dRe t + i dF/dIm t (Eq. 2) scaled by the incoming
gradient; when the probe requires a gradient the same launch also sums
dF/dP = sum_i chi_0 conj(t_0[window]).  Gradients with respect to positions or
measurements are not provided.

``amplitude_loss_potential(ctx, V, sigma, probe, pos, meas)`` is the same cost
of a real potential V with slices t = exp(i sigma V) (Section II-B: V is the
scattering potential); the transmission and the chain rule
dF/dV = sigma Im(conj(t) dF/dt) run in the library's elementwise kernels.
"""
from __future__ import annotations

import torch

from . import _binding as B


class _AmplitudeLoss(torch.autograd.Function):
    @staticmethod
    def forward(fctx, obj, probe, pos, meas, lib_ctx):
        loss = B.ptycho_loss(lib_ctx, obj.detach(), probe.detach(), pos, meas.detach())
        fctx.save_for_backward(obj, probe, pos, meas)
        fctx.lib_ctx = lib_ctx
        return loss.view(())

    @staticmethod
    def backward(fctx, grad_out):
        obj, probe, pos, meas = fctx.saved_tensors
        if fctx.needs_input_grad[3]:
            raise RuntimeError("amplitude_loss differentiates with respect to the object and the probe only")
        grad = pgrad = None
        if fctx.needs_input_grad[0] or fctx.needs_input_grad[1]:
            scale = grad_out.detach().to(torch.float64).reshape(1).contiguous()
            if fctx.needs_input_grad[1]:
                pgrad = torch.empty_like(probe)
            _, grad = B.ptycho_loss_grad(fctx.lib_ctx, obj.detach(), probe.detach(), pos, meas.detach(),
                                         grad_scale=scale, probe_grad=pgrad)
            if not fctx.needs_input_grad[0]:
                grad = None
        return grad, pgrad, None, None, None


def amplitude_loss(lib_ctx: B.Context, obj: torch.Tensor, probe: torch.Tensor, pos: torch.Tensor,
                   meas: torch.Tensor) -> torch.Tensor:
    """F(V) = sum_i sum_q (|G(p_i, V)| - sqrt(meas_i))^2 with a fused-kernel adjoint for autograd."""
    return _AmplitudeLoss.apply(obj, probe, pos, meas, lib_ctx)


class _AmplitudeLossPotential(torch.autograd.Function):
    @staticmethod
    def forward(fctx, V, sigma, probe, pos, meas, lib_ctx):
        t = B.ptycho_potential_transmission(lib_ctx, V.detach(), sigma)
        loss = B.ptycho_loss(lib_ctx, t, probe.detach(), pos, meas.detach())
        fctx.save_for_backward(t, probe, pos, meas)
        fctx.sigma, fctx.lib_ctx = float(sigma), lib_ctx
        return loss.view(())

    @staticmethod
    def backward(fctx, grad_out):
        t, probe, pos, meas = fctx.saved_tensors
        if fctx.needs_input_grad[2] or fctx.needs_input_grad[4]:
            raise RuntimeError("amplitude_loss_potential differentiates with respect to the potential only")
        grad = None
        if fctx.needs_input_grad[0]:
            scale = grad_out.detach().to(torch.float64).reshape(1).contiguous()
            _, gt = B.ptycho_loss_grad(fctx.lib_ctx, t, probe.detach(), pos, meas.detach(), grad_scale=scale)
            grad = B.ptycho_potential_gradient(fctx.lib_ctx, t, gt, fctx.sigma)
        return grad, None, None, None, None, None


def amplitude_loss_potential(lib_ctx: B.Context, V: torch.Tensor, sigma: float, probe: torch.Tensor,
                             pos: torch.Tensor, meas: torch.Tensor) -> torch.Tensor:
    """F(exp(i sigma V)) for a float32 [S, H, W] potential V, differentiable with respect to V."""
    return _AmplitudeLossPotential.apply(V, sigma, probe, pos, meas, lib_ctx)
