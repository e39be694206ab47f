"""torch.autograd.Function around the rasterizer's forward and backward calls.

The forward runs gs_render_fwd and keeps the library frame; the backward runs
gs_render_bwd (reverse traversal, recomputed transmittance) with the incoming
image gradients.  Parameters are passed as the five SoA tensors.
"""
from __future__ import annotations

import torch

from . import core


class RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx_, means, log_scales, quats, opacity_logits, sh, sh_degree, lib_ctx, cams,
                tile, lds_depth, bg):
        params = core.Params(means.detach(), log_scales.detach(), quats.detach(),
                             opacity_logits.detach(), sh.detach(), sh_degree)
        images, frame = core.render_fwd(lib_ctx, params, cams, tile=tile, lds_depth=lds_depth,
                                        bg=bg)
        ctx_.lib_ctx = lib_ctx
        ctx_.frame = frame
        ctx_.params = params
        return torch.stack(images, 0) if len({(c.width, c.height) for c in cams}) == 1 \
            else tuple(images)

    @staticmethod
    def backward(ctx_, *grads):
        g = grads[0]
        dl = [g[i].contiguous() for i in range(g.shape[0])] if len(grads) == 1 and g.dim() == 4 \
            else [x.contiguous() for x in grads]
        out = core.render_bwd(ctx_.lib_ctx, ctx_.frame, ctx_.params, dl)
        return (out.means, out.log_scales, out.quats, out.opacity_logits, out.sh,
                None, None, None, None, None, None)


def rasterize(lib_ctx, params_tensors, sh_degree, cams, *, tile=16, lds_depth=256,
              bg=(0.0, 0.0, 0.0)):
    """Differentiable render of the views in ``cams``: (V, 3, H, W) when the views
    share a size, else a tuple of (3, H_v, W_v)."""
    m, s, q, o, sh = params_tensors
    return RasterizeFn.apply(m, s, q, o, sh, sh_degree, lib_ctx, list(cams), tile, lds_depth,
                             tuple(bg))
