"""torch.autograd wrappers for the transforms (gradients, Sec. 5).

The inverse spin SHT is linear in the coefficients, so its vector-Jacobian
product is the Hermitian adjoint applied to the incoming cotangent (Eqs. 56-58
in the conjugate convention PyTorch uses for complex tensors).  The backward
pass therefore calls the library's dedicated adjoint transform, which
recomputes the Wigner-d functions on the fly instead of storing them.
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
