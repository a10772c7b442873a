"""torch.autograd.Function over libnnm's SIREN value + analytic gradient.

``SirenFn.apply(x, params, d_in, width, n_sine)`` returns (N(x), grad_x N(x)),
both from the fused HIP forward.  Its backward takes upstream adjoints of both
outputs and returns dL/dx and dL/dparams from libnnm's hand-written reverse
mode through primal and tangent (the double backward a gradient-based loss
such as the eikonal term needs).  Only x and params are saved: the backward
recomputes the forward instead of storing activations.
"""

import torch

from . import _binding as B


class SirenFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, params, d_in, width, n_sine):
        x = x.contiguous()
        params = params.contiguous()
        value, grad = B.siren_forward_tangent(d_in, width, n_sine, params, x)
        ctx.save_for_backward(x, params)
        ctx.net = (d_in, width, n_sine)
        return value, grad

    @staticmethod
    def backward(ctx, dvalue, dgrad):
        x, params = ctx.saved_tensors
        dv = dvalue.contiguous() if dvalue is not None else None
        dg = dgrad.contiguous() if dgrad is not None else None
        dx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        dparams, dx = B.siren_backward(*ctx.net, params, x, dv, dg, dx=dx)
        return dx, dparams, None, None, None


def siren(x, params, d_in, width, n_sine):
    """(N(x), grad_x N(x)) differentiable w.r.t. x and params."""
    return SirenFn.apply(x, params, d_in, width, n_sine)
