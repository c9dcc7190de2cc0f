"""The integrator as a differentiable PyTorch function of the integrand's
parameters.

``integral(theta, family, d, rel_tol)`` returns the estimates I(theta_b) of
a batch of parameter vectors. When theta requires a gradient, the forward
run also accumulates, over the partition each integral converges on, the
derivative of the estimate with respect to the parameters (the adjoint of
the estimate: a sum of degree-7 rule values of fixed regions is a weighted
sum of f at fixed points, so its derivative is the same weighted sum of
df/dtheta, computed by the library's adjoint kernel on the GPU). The
backward pass scales those derivatives by the incoming gradient. Without
a gradient the forward run is the plain batched solve.
"""
from __future__ import annotations

import torch

from . import api


class PaganiIntegral(torch.autograd.Function):
    """I(theta) per row of theta [B, n_params]; differentiable in theta."""

    @staticmethod
    def forward(fctx, theta, context, family, d, rel_tol, options):
        th = theta.detach().to("cpu", torch.float64).contiguous().numpy()
        if fctx.needs_input_grad[0]:
            res, G, _ = context.integrate_batch_grad(family, d, th, rel_tol, **options)
            fctx.save_for_backward(torch.as_tensor(G, dtype=theta.dtype,
                                                   device=theta.device))
        else:
            res = context.integrate_batch(family, d, th, rel_tol, **options)
        fctx.results = res
        return torch.tensor([r.estimate for r in res], dtype=theta.dtype,
                            device=theta.device)

    @staticmethod
    def backward(fctx, grad_out):
        (G,) = fctx.saved_tensors
        return grad_out[:, None] * G, None, None, None, None, None


def integral(theta: torch.Tensor, family: str, d: int, rel_tol=1e-3,
             context: api.Context | None = None, **options) -> torch.Tensor:
    """Estimates of the integrals of `family` over [lo, hi] (options lo, hi;
    default the unit cube) for every parameter vector in theta ([B, n] or
    [n]); rel_tol a scalar or [B]. Other options as Context.integrate_batch.
    The estimates are differentiable in theta."""
    if context is None:
        context = api.context(dim_max=d)
    squeeze = theta.dim() == 1
    th = theta[None, :] if squeeze else theta
    out = PaganiIntegral.apply(th, context, family, d, rel_tol, options)
    return out[0] if squeeze else out
