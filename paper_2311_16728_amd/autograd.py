"""torch.autograd.Function over libgs: render (Eq. 3) with a recompute backward.

The forward runs gs_preprocess -> gs_bin_sort -> gs_render_fwd and keeps only
what the rasteriser leaves in the plan's workspaces: projection records, sorted
tile lists, the final transmittance and the restart index of every pixel
(8 bytes per pixel); no per-pixel list of Gaussians is stored.  The backward
calls gs_raster_bwd (which recomputes compositing back to front from those)
and gs_project_bwd.  One forward may be in flight per RenderPlan: a second
forward on the same plan overwrites the saved state.
"""

from __future__ import annotations

import torch

from . import gs
from .mapper import RenderPlan


class GaussianRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, plan: RenderPlan, n: int):
        if params.dtype != torch.float32 or not params.is_contiguous() or params.shape[0] != 59:
            raise ValueError("params must be a contiguous float32 [59, n_cap] tensor")
        plan.render(params, n)
        ctx.plan = plan
        ctx.n = n
        ctx.save_for_backward(params)
        return plan.rgb.clone()

    @staticmethod
    def backward(ctx, grad_rgb: torch.Tensor):
        (params,) = ctx.saved_tensors
        plan: RenderPlan = ctx.plan
        grad = torch.zeros_like(params)
        g = grad_rgb.contiguous()
        gs.gs_raster_bwd(plan.settings, plan.proj_ws, plan.n_cap, plan.n_views, plan.sort_ws,
                         plan.pair_cap, plan.targets_dev, plan.n_targets, plan.total_tiles, plan.T,
                         plan.last, g, plan.accum_ws)
        gs.gs_project_bwd(plan.settings, params, ctx.n, plan.views_dev, plan.n_views, plan.accum_ws,
                          grad)
        return grad, None, None


def render(params: torch.Tensor, plan: RenderPlan, n: int) -> torch.Tensor:
    """Differentiable render of every target of `plan`; returns the packed planar images."""
    return GaussianRender.apply(params, plan, n)


def saved_state_bytes(plan: RenderPlan) -> int:
    """Bytes the backward needs beyond the parameters: records, sorted lists,
    per-pixel final transmittance and restart index, 2D-gradient accumulators."""
    s = plan.sizes
    return int(s.proj_bytes + s.sort_bytes + s.accum_bytes + 8 * plan.total_pixels)
