"""torch.autograd bindings: NLL -> gradient -> Hessian-vector product.

NLLFunction.forward runs pwa_nll; its backward is GradFunction (pwa_grad),
whose backward is pwa_hvp.  So `torch.autograd.grad(nll, theta,
create_graph=True)` gives the hand-written adjoint gradient and a second
`torch.autograd.grad(g @ v, theta)` gives the forward-over-reverse H v,
with no per-event tape: each call is one pass over the bound events.
"""

import torch


class GradFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, lik):
        _, g = lik.grad(theta.detach())
        ctx.save_for_backward(theta)
        ctx.lik = lik
        return g.clone()

    @staticmethod
    def backward(ctx, gv):
        (theta,) = ctx.saved_tensors
        hv, _, _ = ctx.lik.hvp(theta.detach(), gv.detach().contiguous())
        return hv.clone(), None


class NLLFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, lik):
        ctx.save_for_backward(theta)
        ctx.lik = lik
        return lik.nll(theta.detach()).clone()

    @staticmethod
    def backward(ctx, gout):
        (theta,) = ctx.saved_tensors
        return gout * GradFunction.apply(theta, ctx.lik), None


def nll(theta, lik):
    """Differentiable NLL(theta) (twice: gradient and Hessian-vector products)."""
    return NLLFunction.apply(theta, lik)
