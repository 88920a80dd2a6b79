"""Gradient-driven densification for a Mapper (Section 3.3.1: split or clone
primitives with large loss gradients, as 3D Gaussian splatting does, and
prune faint or oversized ones).

``Densifier`` owns the statistic ([2][n_cap]), the split noise, the output
buffers and the workspace; every step runs in libgs (gs_densify_stats,
gs_densify, gs_reset_opacity).  After a densification the mapper's
parameter and moment tensors are exchanged with the output buffers (the
previous tensors become the next call's outputs), its count changes and its
version is bumped, so render plans re-project and captured graphs must be
captured again.
"""

from __future__ import annotations

import torch

from . import gs


class Densifier:
    def __init__(self, mapper, extent: float, grad_threshold: float = 2e-4, percent_dense: float = 0.01,
                 min_opacity: float = 0.005, big_fraction: float | None = 0.1, seed: int = 0):
        self.mapper = mapper
        self.rule = gs.densify_rule(extent, grad_threshold, percent_dense, min_opacity, big_fraction)
        p = mapper.params
        self.n_cap = p.shape[1]
        dev = p.device
        self.stats = torch.zeros(2, self.n_cap, dtype=torch.float32, device=dev)
        self.noise = torch.zeros(6, self.n_cap, dtype=torch.float32, device=dev)
        self.out = [torch.zeros_like(p), torch.zeros_like(p), torch.zeros_like(p)]
        self.ws = torch.empty(gs.gs_densify_workspace_bytes(self.n_cap), dtype=torch.uint8, device=dev)
        self.counts = torch.zeros(4, dtype=torch.int64, device=dev)
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)

    def accumulate(self, plan, stream=None):
        """Adds the backward pass just run on `plan` to the statistic."""
        if plan.n_cap != self.n_cap:
            raise gs.GsError("the plan's column capacity differs from the parameters'")
        gs.gs_densify_stats(plan.accum_ws, self.mapper.n, self.n_cap, plan.views_dev, plan.n_views,
                            self.stats, stream)

    def densify(self, stream=None) -> dict:
        """Applies the rule, swaps in the result and restarts the statistic.
        Returns the counts (synchronises)."""
        mp = self.mapper
        self.noise.normal_(generator=self.gen)
        gs.gs_densify(self.rule, mp.params, mp.m, mp.v, self.stats, self.noise, mp.n, self.out[0],
                      self.out[1], self.out[2], self.ws, self.counts, stream)
        n_out, cloned, split, pruned = (int(x) for x in self.counts.cpu())
        if n_out > self.n_cap:
            raise gs.GsError(f"densification needs {n_out} columns, capacity is {self.n_cap}")
        old = [mp.params, mp.m, mp.v]
        mp.params, mp.m, mp.v = self.out
        self.out = old
        mp.n = n_out
        mp.invalidate()
        gs.gs_fill(self.stats, 0.0, stream)
        return dict(n_out=n_out, cloned=cloned, split=split, pruned=pruned)

    def reset_opacity(self, max_opacity: float = 0.01, stream=None):
        mp = self.mapper
        gs.gs_reset_opacity(mp.params, mp.m, mp.v, mp.n, max_opacity, stream)
        mp.invalidate()
