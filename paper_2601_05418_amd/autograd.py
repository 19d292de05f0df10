"""Differentiable compressed encoding for learned / unrolled reconstruction.

`Encode` is E' (forward) with E'^H as its backward, `Adjoint` the reverse,
`GDStep` one gradient step x - alpha (E'^H E' x - b) with gradients for x, b
and the real step size alpha, and `UnrolledGD` a fixed number of such steps
with one learnable step size each, checkpointed every few steps so that
only the segment inputs are kept during the forward pass.  Every operator
application and every update runs in libgpjc's kernels; these classes only
pass tensors through (PyTorch's conjugate-Wirtinger convention: for a real
loss, the gradient of a linear map A is A^H applied to the upstream one).
"""
from __future__ import annotations

import torch
from torch.utils.checkpoint import checkpoint

from . import gpjc


def _c64(t):
    return t.to(torch.complex64)  # the binding materialises conj / neg views


class Encode(torch.autograd.Function):
    """y = E' x (the plan's forward), backward E'^H."""

    @staticmethod
    def forward(ctx, x, plan, prec="fp32"):
        ctx.plan, ctx.prec = plan, prec
        return plan.forward(_c64(x), prec=prec)

    @staticmethod
    def backward(ctx, gy):
        return ctx.plan.adjoint(_c64(gy), prec=ctx.prec), None, None


class Adjoint(torch.autograd.Function):
    """x = E'^H y, backward E'."""

    @staticmethod
    def forward(ctx, y, plan, prec="fp32"):
        ctx.plan, ctx.prec = plan, prec
        return plan.adjoint(_c64(y), prec=prec)

    @staticmethod
    def backward(ctx, gx):
        return ctx.plan.forward(_c64(gx), prec=ctx.prec), None, None


class GDStep(torch.autograd.Function):
    """x_out = x - alpha (E'^H E' x - b); alpha a 0-d float32 tensor."""

    @staticmethod
    def forward(ctx, x, b, alpha, plan, prec="fp32"):
        xo, r = plan.gd_step(_c64(x), _c64(b), alpha.reshape(1), prec=prec)
        ctx.plan, ctx.prec = plan, prec
        ctx.save_for_backward(alpha, r)
        return xo

    @staticmethod
    def backward(ctx, g):
        alpha, r = ctx.saved_tensors
        gx, gb, ga = ctx.plan.gd_step_backward(_c64(g), alpha.reshape(1), r, prec=ctx.prec,
                                               want_gx=ctx.needs_input_grad[0], want_gb=ctx.needs_input_grad[1])
        return gx, gb, ga.reshape(alpha.shape).to(alpha.dtype), None, None


class UnrolledGD(torch.nn.Module):
    """`steps` gradient steps on 1/2 ||E' x - y||^2 from x0 (zeros by
    default), step k with its own learnable size alpha_k (initialised to
    alpha0, e.g. 1/L).  `checkpoint_every` > 0 recomputes each segment of
    that many steps in the backward pass instead of keeping its residuals."""

    def __init__(self, plan, steps=10, alpha0=1.0, checkpoint_every=2, prec="fp32"):
        super().__init__()
        self.plan, self.steps, self.prec = plan, int(steps), prec
        self.checkpoint_every = int(checkpoint_every)
        self.alpha = torch.nn.Parameter(torch.full((self.steps,), float(alpha0), dtype=torch.float32,
                                                   device=plan.device))

    def _segment(self, x, b, k0, k1):
        for k in range(k0, k1):
            x = GDStep.apply(x, b, self.alpha[k], self.plan, self.prec)
        return x

    def forward(self, y, x0=None):
        b = Adjoint.apply(y, self.plan, self.prec)
        x = torch.zeros(self.plan.image_shape(), dtype=torch.complex64, device=self.plan.device) if x0 is None \
            else x0
        seg = self.checkpoint_every if self.checkpoint_every > 0 else self.steps
        for k0 in range(0, self.steps, seg):
            k1 = min(self.steps, k0 + seg)
            if self.checkpoint_every > 0 and torch.is_grad_enabled():
                x = checkpoint(self._segment, x, b, k0, k1, use_reentrant=False)
            else:
                x = self._segment(x, b, k0, k1)
        return x
