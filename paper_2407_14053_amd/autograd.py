"""torch.autograd.Function around the DirectL forward/backward of the C ABI (marshalling only: both passes run
in the gfx950 kernels).  Parameters are the user-layout tensors (means[G,3], log_scales[G,3], quats[G,4],
opacity_logits[G], sh[G,16,3]); the output is the encoded image [H,W,3]."""
from __future__ import annotations

import torch

from . import api


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, rnd, c2w, means, log_scales, quats, logits, sh):
        params = (means, log_scales, quats, logits, sh)
        rnd.scene.update(params)
        out = api.render(rnd.ctx, rnd.scene, rnd.display, c2w, opts=rnd.opts)
        fctx.rnd = rnd
        fctx.c2w = c2w
        fctx.save_for_backward(means, log_scales, quats, logits, sh, out)
        return out

    @staticmethod
    def backward(fctx, grad_out):
        means, log_scales, quats, logits, sh, out = fctx.saved_tensors
        rnd = fctx.rnd
        # the scene may have been updated by a later forward: upload the parameters of this one
        rnd.scene.update((means, log_scales, quats, logits, sh))
        g = api.render_backward(rnd.ctx, rnd.scene, rnd.display, fctx.c2w, out, grad_out, opts=rnd.opts)
        return (None, None) + tuple(g)


class LightFieldRenderer:
    """Differentiable light-field renderer for one display.  ``render(params, c2w)`` returns the encoded image;
    gradients flow to the five parameter tensors."""

    def __init__(self, ctx: api.Context, display, n_gaussians: int, opts=None):
        self.ctx = ctx
        self.display = display if isinstance(display, api.Display) else api.Display(ctx, display)
        self.opts = opts or api.default_opts()
        dev = dict(dtype=torch.float32, device="cuda")
        init = (torch.zeros((n_gaussians, 3), **dev), torch.zeros((n_gaussians, 3), **dev),
                torch.tensor([1.0, 0, 0, 0], **dev).repeat(n_gaussians, 1), torch.zeros((n_gaussians,), **dev),
                torch.zeros((n_gaussians, 16, 3), **dev))
        self.scene = api.Scene(ctx, init)

    def render(self, params, c2w):
        return _RenderFn.apply(self, c2w, *params)
