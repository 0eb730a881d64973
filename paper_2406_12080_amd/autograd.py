"""``torch.autograd.Function`` over the library's render / render_backward.

The forward renders every view in one call (one graph launch for several
views); the backward hands dL/dimage to ``hgs_render_backward``, which
returns gradients for every interior node's parameters (leaves are frozen)
through the parent/child interpolation and the opacity transition.

The renderer keeps the state of its last render only: each node of the
autograd graph records the id of its render, and its backward fails with
HGS_ERR_STATE when a later render on the same renderer has replaced that
state (differentiate before rendering again, or use one renderer per
render that stays in the graph).
"""
from __future__ import annotations

import torch

from .hgs import PARAM_FIELDS, Renderer


class HierRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer: Renderer, views, mean, scale, rot, opacity, sh):
        params = (mean, scale, rot, opacity, sh)
        renderer.bind(*params)
        imgs, stats = renderer.render(views)
        ctx.renderer = renderer
        ctx.render_id = stats["render_id"]
        ctx.shapes = [p.shape for p in params]
        ctx.stats = stats
        ctx.out_shapes = [i.shape for i in imgs]
        return tuple(imgs)

    @staticmethod
    def backward(ctx, *grad_imgs):
        r: Renderer = ctx.renderer
        dev = r.device
        grads = {k: torch.zeros(s, dtype=torch.float32, device=dev) for k, s in zip(PARAM_FIELDS, ctx.shapes)}
        dL = [g if g is not None else torch.zeros(s, dtype=torch.float32, device=dev)
              for g, s in zip(grad_imgs, ctx.out_shapes)]
        r.backward(dL, grads, render_id=ctx.render_id)
        return (None, None) + tuple(grads[k] for k in PARAM_FIELDS)


def render(renderer: Renderer, views, params: dict):
    """Differentiable render of ``views``; ``params`` maps the five parameter
    names to CUDA tensors (leaves of the autograd graph)."""
    return HierRender.apply(renderer, list(views), *[params[k] for k in PARAM_FIELDS])
