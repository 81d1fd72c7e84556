"""torch.autograd wrappers of the HIP operators.

ConvectiveFn: forward = dg_apply_convective, backward = dg_vjp_convective
(the hand-written adjoint kernel).  LaplaceFn: the SIPG form is symmetric, so
its backward is the forward apply of the incoming gradient.  Gradients are
produced by the GPU kernels only; there is no fallback path.
"""
import torch

from . import dgmf


class ConvectiveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, desc):
        u = u.contiguous()
        ctx.save_for_backward(u)
        ctx.desc = desc
        return dgmf.apply_convective(desc, u)

    @staticmethod
    def backward(ctx, grad_out):
        (u,) = ctx.saved_tensors
        g = dgmf.vjp_convective(ctx.desc, u, grad_out.contiguous().to(u.dtype))
        return g, None


class LaplaceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, desc):
        ctx.desc = desc
        return dgmf.apply_laplace(desc, u.contiguous())

    @staticmethod
    def backward(ctx, grad_out):
        return dgmf.apply_laplace(ctx.desc, grad_out.contiguous()), None


def convective(u, degree, n_el, length=None, lf_factor=1.0):
    """Differentiable convective residual R(u); u: [3, N_el, (k+1)^3] on the GPU."""
    return ConvectiveFn.apply(u, dgmf.make_desc(degree, n_el, length, lf_factor=lf_factor))


def laplace(u, degree, n_el, length=None, penalty_factor=1.0, scale=1.0):
    """Differentiable SIPG Laplace apply; u: [N_el, n^3] or [3, N_el, n^3]."""
    n_comp = 3 if u.dim() == 3 else 1
    desc = dgmf.make_desc(degree, n_el, length, penalty_factor=penalty_factor, scale=scale, n_comp=n_comp)
    return LaplaceFn.apply(u, desc)
