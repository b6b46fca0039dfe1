"""torch.autograd wrappers for the spin SHTs and Wigner transforms (gradients, Sec. 5).

Both transforms are linear, so each vector-Jacobian product is the Hermitian
adjoint applied to the incoming cotangent (Eqs. 56-58 in the conjugate
convention PyTorch uses for complex tensors), and each Jacobian-vector
product (forward-mode AD) is the transform itself applied to the tangent.
The backward passes call the library's dedicated adjoint transforms, which
recompute the Wigner-d functions on the fly instead of storing them: the
adjoint of the inverse is a forward-type sweep, the adjoint of the forward an
inverse-type sweep.
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

    @staticmethod
    def jvp(ctx, t_flm, t_plan):
        return ctx.plan.inverse(t_flm.contiguous())


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

    @staticmethod
    def jvp(ctx, t_f, t_plan):
        return ctx.plan.forward(t_f.contiguous())


def forward(f, plan):
    """Differentiable forward spin SHT: map -> flm [B?, L, 2L-1] (FP64 plans)."""
    if not isinstance(plan, binding.Plan):
        raise TypeError("plan must be a paper_2311_14670_amd.binding.Plan")
    return _S2Forward.apply(f, plan)


class _SO3Inverse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, flmn, plan):
        ctx.plan = plan
        return plan.so3_inverse(flmn)

    @staticmethod
    def backward(ctx, grad_f):
        if not ctx.needs_input_grad[0]:
            return None, None
        return ctx.plan.so3_inverse_adjoint(grad_f.contiguous()), None

    @staticmethod
    def jvp(ctx, t_flmn, t_plan):
        return ctx.plan.so3_inverse(t_flmn.contiguous())


def so3_inverse(flmn, plan):
    """Differentiable inverse Wigner transform: flmn [B?, 2N-1, L, 2L-1] -> f."""
    if not isinstance(plan, binding.Plan):
        raise TypeError("plan must be a paper_2311_14670_amd.binding.Plan")
    return _SO3Inverse.apply(flmn, plan)


class _SO3Forward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        return plan.so3_forward(f)

    @staticmethod
    def backward(ctx, grad_flmn):
        if not ctx.needs_input_grad[0]:
            return None, None
        return ctx.plan.so3_forward_adjoint(grad_flmn.contiguous()), None

    @staticmethod
    def jvp(ctx, t_f, t_plan):
        return ctx.plan.so3_forward(t_f.contiguous())


def so3_forward(f, plan):
    """Differentiable forward Wigner transform: f [B?, 2N-1, L, 2L-1] -> flmn (FP64 plans)."""
    if not isinstance(plan, binding.Plan):
        raise TypeError("plan must be a paper_2311_14670_amd.binding.Plan")
    return _SO3Forward.apply(f, plan)


class _S2InverseReal(torch.autograd.Function):
    @staticmethod
    def forward(ctx, flm, plan):
        ctx.plan = plan
        return plan.inverse_real(flm)

    @staticmethod
    def backward(ctx, grad_f):
        if not ctx.needs_input_grad[0]:
            return None, None
        return ctx.plan.inverse_real_adjoint(grad_f.contiguous()), None

    @staticmethod
    def jvp(ctx, t_flm, t_plan):
        return ctx.plan.inverse_real(t_flm.contiguous())


def inverse_real(flm, plan):
    """Differentiable real-signal inverse SHT (spin 0): flm [B?, L, 2L-1] complex128,
    orders m >= 0 used -> real map.  The orders m < 0 get zero gradient."""
    if not isinstance(plan, binding.Plan):
        raise TypeError("plan must be a paper_2311_14670_amd.binding.Plan")
    return _S2InverseReal.apply(flm, plan)


class _S2ForwardReal(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        return plan.forward_real(f)

    @staticmethod
    def backward(ctx, grad_flm):
        if not ctx.needs_input_grad[0]:
            return None, None
        return ctx.plan.forward_real_adjoint(grad_flm.contiguous()), None

    @staticmethod
    def jvp(ctx, t_f, t_plan):
        return ctx.plan.forward_real(t_f.contiguous())


def forward_real(f, plan):
    """Differentiable forward SHT of a real map (spin 0): float64 map -> flm."""
    if not isinstance(plan, binding.Plan):
        raise TypeError("plan must be a paper_2311_14670_amd.binding.Plan")
    return _S2ForwardReal.apply(f, plan)
