"""``torch.autograd`` face of the renderer: the forward is ``dvgo_render_fwd``,
the backward is the library's recompute-from-the-end adjoint
``dvgo_render_bwd``: the derivative of the colour quadrature of the
Preliminaries section (Eq. volume_rendering) and of the fine-stage queries
(Eq. fine_queries), written out by hand with no per-sample state saved.

Only per-ray tensors (log T at the ray end) and the sample list survive
between the two calls.  Arguments are marshalled here; every computation
runs in the library.
"""

from __future__ import annotations

from typing import Optional

import torch

from . import api
from ._lib import DVGO_F32


class RenderFn(torch.autograd.Function):
    """(density [nx,ny,nz], feat [nx,ny,nz,12], mlp_flat [22019]) -> (rgb [B,3], depth [B], acc [B]).

    Gradients come back dense and float32: grid gradients in the grids'
    shapes (also when features are read from a bfloat16 shadow) and the flat
    network gradient.  The sample list ``s`` fixes which points are
    evaluated; it is not differentiated."""

    @staticmethod
    def forward(ctx, density, feat, mlp_flat, s: api.Samples, box_min, box_max, act_shift: float, bg,
                precision: int, feat_shadow: Optional[torch.Tensor]):
        grid = api.Grid(density, feat, tuple(box_min), tuple(box_max), float(act_shift))
        grid.feat_shadow = feat_shadow
        out = api.render_fwd(grid, mlp_flat, s, bg, precision=precision, use_shadow=feat_shadow is not None,
                             want_depth_acc=True)
        ctx.save_for_backward(density, feat, mlp_flat, out["log_t_end"])
        ctx.s, ctx.bg, ctx.precision, ctx.feat_shadow = s, bg, precision, feat_shadow
        ctx.geom = (tuple(box_min), tuple(box_max), float(act_shift))
        ctx.set_materialize_grads(False)
        return out["rgb"], out["depth"], out["acc"]

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_acc):
        density, feat, mlp_flat, log_t_end = ctx.saved_tensors
        grid = api.Grid(density, feat, *ctx.geom)
        grid.feat_shadow = ctx.feat_shadow
        if g_rgb is None:
            g_rgb = torch.zeros((ctx.s.B, 3), dtype=torch.float32, device=density.device)
        gd = torch.zeros_like(density)
        gf = torch.zeros(feat.shape, dtype=torch.float32, device=feat.device)
        gm = torch.zeros_like(mlp_flat)
        api.render_bwd(grid, mlp_flat, ctx.s, log_t_end, g_rgb.contiguous(), gd, gf, gm, ctx.bg,
                       precision=ctx.precision, use_shadow=ctx.feat_shadow is not None,
                       grad_depth=None if g_depth is None else g_depth.contiguous(),
                       grad_acc=None if g_acc is None else g_acc.contiguous())
        return gd, gf, gm, None, None, None, None, None, None, None


def render(density, feat, mlp_flat, s: api.Samples, box_min, box_max, act_shift: float, bg=(1.0, 1.0, 1.0),
           precision: int = DVGO_F32, feat_shadow: Optional[torch.Tensor] = None):
    """Differentiable colour, depth and opacity of the rays in ``s``."""
    return RenderFn.apply(density, feat, mlp_flat, s, box_min, box_max, act_shift, bg, precision, feat_shadow)
