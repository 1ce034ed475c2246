"""torch.autograd glue for direct fine-tuning of the leaf coefficients (Sec. 4.3).

The forward and backward passes are libfpo calls (fpo_render_rays and
fpo_render_backward); the optimiser step is fpo_adam_step.  Nothing here
computes on tensors itself: a caller writes the loss of Eq. 13 (or any other
loss of the rendered colours) with torch, calls loss.backward(), and the
library's backward kernel scatters dL/drgb into the coefficient records.

    coeffs = tree.coeffs.requires_grad_()
    opt = Adam(coeffs, lr=1e-2)
    rgb = render(tree, o, d, t_idx, basis, opts)
    ((rgb - target) ** 2).sum(1).mean().backward()
    opt.step()                       # uses and clears coeffs.grad
"""
from __future__ import annotations

from typing import Optional

import torch

from . import _lib


class FPORender(torch.autograd.Function):
    """rgb = render(coeffs) for given rays; coeffs are the F32 leaf records
    of `tree` (passed explicitly so that autograd tracks them).  With
    FPO_RAYS_RECORD in opts the forward's segment records in opts.workspace
    serve the backward, so the same opts must not be reused for another
    forward before backward() runs."""

    @staticmethod
    def forward(ctx, coeffs, tree: _lib.DeviceTree, o, d, t_idx, basis, opts: _lib.RenderOpts):
        if coeffs.data_ptr() != tree.coeffs.data_ptr():
            raise ValueError("coeffs must be the tree's coefficient store")
        rgb, _ = _lib.render_rays(tree, o, d, t_idx, basis, opts)
        ctx.save_for_backward(o, d, t_idx, basis, rgb)
        ctx.tree = tree
        ctx.opts = opts
        return rgb

    @staticmethod
    def backward(ctx, grad_rgb):
        o, d, t_idx, basis, rgb = ctx.saved_tensors
        grad = torch.zeros_like(ctx.tree.coeffs)
        _lib.render_backward(ctx.tree, o, d, t_idx, basis, rgb, grad_rgb.contiguous(), grad, ctx.opts)
        return grad, None, None, None, None, None, None


def render(tree: _lib.DeviceTree, o, d, t_idx, basis, opts: Optional[_lib.RenderOpts] = None):
    """Colours [n][3] of rays (o, d) at basis rows t_idx, differentiable in
    tree.coeffs."""
    return FPORender.apply(tree.coeffs, tree, o, d, t_idx, basis, opts or _lib.make_opts())


class Adam:
    """Adam over a flat float tensor (the coefficient records), one fused
    fpo_adam_step per step; the gradient buffer is cleared by the step."""

    def __init__(self, params: torch.Tensor, lr: float = 1e-2, betas=(0.9, 0.999), eps: float = 1e-8):
        self.params = params
        self.m = torch.zeros_like(params, requires_grad=False)
        self.v = torch.zeros_like(params, requires_grad=False)
        self.lr = float(lr)
        self.betas = (float(betas[0]), float(betas[1]))
        self.eps = float(eps)
        self.t = 0

    def step(self, grad: Optional[torch.Tensor] = None):
        """One update with `grad`, or with params.grad (left by backward())."""
        if grad is None:
            grad = self.params.grad
            if grad is None:
                raise RuntimeError("no gradient: call backward() first or pass grad")
        self.t += 1
        with torch.no_grad():
            _lib.adam_step(self.params, grad, self.m, self.v, self.t, self.lr, self.betas[0], self.betas[1],
                           self.eps)
