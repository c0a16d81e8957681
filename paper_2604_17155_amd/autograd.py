"""torch.autograd.Function wrappers of colorize and render.

Gradients flow to the targets and the opacities only (the geometry is held
fixed, as in the paper's setting of a trained splat scene).  The backward
passes call the hand-written adjoints gsc_colorize_backward and
gsc_render_backward, which recompute the per-pixel weights instead of storing
them.

Every call bins the scene again unless the caller passes reuse_binning=True.
Then a call on the same tensor objects, with unchanged torch versions and the
same cameras, reuses the previous call's tile lists and skips the projection.
Only the caller knows that no write went round torch's version counter
(`t.data` edits, graph replays, other libraries). After such a write, reused
lists carry the old opacities and geometry.

    coeffs = colorize(targets, opacities, means, scales, quats, cams, sh_deg, lam)
    images = render(coeffs, opacities, means, scales, quats, cams)
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch

from . import gsc

_default_ctx: Optional[gsc.Context] = None


def default_context() -> gsc.Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = gsc.Context()
    return _default_ctx


class ColorizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, targets, opacities, means, scales, quats, cams, sh_deg, lam, context, offsets,
                reuse):
        g = context or default_context()
        coeffs, _ = g.colorize(means, scales, quats, opacities, cams, targets, sh_deg, lam,
                               offsets=offsets, with_status=False, reuse_binning=reuse)
        ctx.save_for_backward(targets, opacities, means, scales, quats, coeffs)
        ctx.cams, ctx.sh_deg, ctx.lam, ctx.g, ctx.offsets = cams, sh_deg, list(lam), g, offsets
        ctx.reuse = reuse
        return coeffs

    @staticmethod
    def backward(ctx, grad_coeffs):
        targets, opacities, means, scales, quats, coeffs = ctx.saved_tensors
        want_t, want_o = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gt = go = None
        if want_t or want_o:
            gt, go = ctx.g.colorize_backward(means, scales, quats, opacities, ctx.cams, targets,
                                             ctx.sh_deg, ctx.lam, coeffs,
                                             grad_coeffs.detach().float().contiguous(),
                                             want_targets=want_t, want_opacities=want_o,
                                             offsets=ctx.offsets, reuse_binning=ctx.reuse)
            if gt is not None and gt.dtype != targets.dtype:
                gt = gt.to(targets.dtype)
        return gt, go, None, None, None, None, None, None, None, None, None


class RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coeffs, opacities, means, scales, quats, cams, context, offsets, reuse):
        g = context or default_context()
        coeffs = coeffs.detach().float().contiguous()
        images = g.render(means, scales, quats, opacities, cams, coeffs, offsets=offsets,
                          reuse_binning=reuse)
        ctx.save_for_backward(coeffs, opacities, means, scales, quats)
        ctx.cams, ctx.g, ctx.offsets, ctx.reuse = cams, g, offsets, reuse
        return images

    @staticmethod
    def backward(ctx, grad_images):
        coeffs, opacities, means, scales, quats = ctx.saved_tensors
        want_c, want_o = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gc = go = None
        if want_c or want_o:
            gc, go = ctx.g.render_backward(means, scales, quats, opacities, ctx.cams, coeffs,
                                           grad_images.detach().float().contiguous(),
                                           want_coeffs=want_c, want_opacities=want_o,
                                           offsets=ctx.offsets, reuse_binning=ctx.reuse)
        return gc, go, None, None, None, None, None, None, None


def colorize(targets, opacities, means, scales, quats, cams: Sequence, sh_deg: int, lam,
             context: Optional[gsc.Context] = None, offsets=None, reuse_binning: bool = False):
    """Differentiable colorize: coeffs [N,(L+1)^2,C] float32.  reuse_binning as
    in the module docstring (off by default)."""
    return ColorizeFn.apply(targets, opacities, means, scales, quats, cams, sh_deg, lam, context,
                            offsets, bool(reuse_binning))


def render(coeffs, opacities, means, scales, quats, cams: Sequence,
           context: Optional[gsc.Context] = None, offsets=None, reuse_binning: bool = False):
    """Differentiable render: images [sum HW, C] float32.  reuse_binning as in
    the module docstring (off by default)."""
    return RenderFn.apply(coeffs, opacities, means, scales, quats, cams, context, offsets,
                          bool(reuse_binning))
