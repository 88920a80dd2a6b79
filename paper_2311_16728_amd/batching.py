"""Batched mapping: every keyframe at every Gaussian-pyramid level in one pass.

Eq. 5 supervises the map with the levels of each keyframe's Gaussian pyramid.
Here all (keyframe, level) targets of an iteration form one RenderPlan, so each
stage is a single launch over all of their tiles (96 targets = 32 keyframes x
3 levels in the benchmark), the parameters are read and updated once per
iteration for all of them, and the whole iteration is captured into one HIP
graph and replayed.  The Adam step count lives in device memory and is
advanced inside the graph.  The ground truth of level l is level l of the
keyframe image's pyramid (gs_pyramid_build), rendered targets use intrinsics
divided by 2^l.
"""

from __future__ import annotations

import numpy as np
import torch

from . import gs
from .mapper import LAMBDA, PYRAMID_LEVELS, RenderPlan


class BatchedMapper:
    def __init__(self, params: torch.Tensor, n: int, cams, gt_images, levels: int = PYRAMID_LEVELS,
                 pair_cap: int = 1 << 28, settings=None, lr_rows=None, lam: float = LAMBDA,
                 beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15, tile_w: int = gs.TILE):
        self.params = params
        self.n = n
        self.levels = levels
        self.lam = lam
        self.beta1, self.beta2, self.eps = beta1, beta2, eps
        self.lr_rows = np.full(59, 1e-3, np.float32) if lr_rows is None else np.asarray(lr_rows, np.float32)
        specs = [(v, l, tuple(np.asarray(c.get("bg", (0, 0, 0)), np.float64)), 1.0)
                 for v, c in enumerate(cams) for l in range(levels)]
        self._plan_args = (cams, specs, params.shape[1], pair_cap)
        self.plan = self.make_plan(tile_w, settings)
        self.target = torch.empty(3 * self.plan.total_pixels, dtype=torch.float32, device=params.device)
        self._build_targets(gt_images)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.d_step = torch.zeros(1, dtype=torch.int32, device=params.device)
        self.graph = None

    def make_plan(self, tile_w: int, settings=None) -> RenderPlan:
        """A render plan over this mapper's targets with tiles tile_w wide (the
        packed image layout, and so the ground truth, does not depend on it);
        assign it to .plan to use it."""
        cams, specs, n_cap, pair_cap = self._plan_args
        return RenderPlan(cams, specs, n_cap, pair_cap, settings, self.params.device, tile_w)

    def _build_targets(self, gt_images):
        """Level l of every keyframe's Gaussian pyramid into its target slot."""
        for v, img in enumerate(gt_images):
            img = img.contiguous()
            sizes = []
            h, w = img.shape[1], img.shape[2]
            for _ in range(self.levels):
                sizes.append((h, w))
                h, w = (h + 1) // 2, (w + 1) // 2
            pyr = torch.empty(sum(3 * a * b for a, b in sizes), dtype=torch.float32, device=img.device)
            gs.gs_pyramid_build(img, self.levels, pyr)
            at = 0
            for l, (h, w) in enumerate(sizes):
                self.plan.image(self.target, v * self.levels + l).copy_(pyr[at:at + 3 * h * w].view(3, h, w))
                at += 3 * h * w

    def invalidate(self):
        """Call after changing the parameters outside iteration() (the next
        iteration then projects again)."""
        self.plan.records_of = None

    def iteration(self, stream=None):
        """One batched iteration: render all targets, Eq. 4 over all targets,
        backward, Adam (step counter advanced on the device).  The optimiser
        step also writes the projection records of the updated parameters, so
        only the first iteration runs gs_preprocess."""
        p = self.plan
        if p.records_of != id(self):
            p.preprocess(self.params, self.n, stream)
        p.bin_sort(self.n, stream)
        p.render_fwd(stream=stream)
        p.loss(self.target, self.lam, True, stream)
        gs.gs_raster_bwd(p.settings, p.proj_ws, p.n_cap, p.n_views, p.sort_ws, p.pair_cap, p.targets_dev,
                         p.n_targets, p.total_tiles, p.T, p.last, p.dL, p.accum_ws, stream)
        gs.gs_step_advance(self.d_step, stream)
        gs.gs_project_bwd_adam(p.settings, self.params, self.n, p.views_dev, p.n_views, p.accum_ws,
                               self.m, self.v, self.lr_rows, self.d_step, self.beta1, self.beta2,
                               self.eps, p.proj_ws, stream)
        p.records_of = id(self)

    def capture(self, warmup: int = 1):
        """Capture one iteration into a HIP graph (after `warmup` eager iterations
        on a side stream, which also advance the optimiser)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                self.iteration()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.iteration()
        # capturing does not run the iteration
        torch.cuda.synchronize()
        return self.graph

    def step(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self.iteration()

    @property
    def step_count(self) -> int:
        return int(self.d_step.item())


def psnr(plan: RenderPlan, rendered: torch.Tensor, target: torch.Tensor) -> float:
    """Mean PSNR over the plan's targets (images clamped to [0, 1])."""
    vals = []
    for i in range(plan.n_targets):
        a = plan.image(rendered, i).clamp(0, 1)
        b = plan.image(target, i).clamp(0, 1)
        mse = float(((a - b) ** 2).mean())
        vals.append(10.0 * np.log10(1.0 / max(mse, 1e-12)))
    return float(np.mean(vals))
