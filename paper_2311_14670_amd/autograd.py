"""torch.autograd wrappers for the transforms (gradients, Sec. 5).

Both transforms are linear, so each vector-Jacobian product is the Hermitian
adjoint applied to the incoming cotangent (Eqs. 56-58 in the conjugate
convention PyTorch uses for complex tensors).  The backward passes call the
library's dedicated adjoint transforms, which recompute the Wigner-d
functions on the fly instead of storing them: the adjoint of the inverse is
a forward-type sweep, the adjoint of the forward an inverse-type sweep.
"""
import torch

from . import binding


class _S2Inverse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, flm, plan):
        ctx.plan = plan
        return plan.inverse(flm)

    @staticmethod
    def backward(ctx, grad_f):
        if not ctx.needs_input_grad[0]:
            return None, None
        return ctx.plan.inverse_adjoint(grad_f.contiguous()), None


def inverse(flm, plan):
    """Differentiable inverse spin SHT: flm [B?, L, 2L-1] complex128 -> map."""
    if not isinstance(plan, binding.Plan):
        raise TypeError("plan must be a paper_2311_14670_amd.binding.Plan")
    return _S2Inverse.apply(flm, plan)


class _S2Forward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        return plan.forward(f)

    @staticmethod
    def backward(ctx, grad_flm):
        if not ctx.needs_input_grad[0]:
            return None, None
        return ctx.plan.forward_adjoint(grad_flm.contiguous()), None


def forward(f, plan):
    """Differentiable forward spin SHT: map -> flm [B?, L, 2L-1] (FP64 plans)."""
    if not isinstance(plan, binding.Plan):
        raise TypeError("plan must be a paper_2311_14670_amd.binding.Plan")
    return _S2Forward.apply(f, plan)
