"""One mapping iteration of the photorealistic mapper, chained from libgs calls.

``RenderPlan`` owns the device descriptors (views, targets) and every
workspace for a fixed problem shape, so that the sequence
preprocess -> bin/sort -> render -> loss -> backward -> Adam allocates nothing
once built and can be captured in a HIP graph.  ``Mapper`` holds the
parameter store and the Adam moments.  Torch is used for device memory and
streams only.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

from . import gs

LAMBDA = 0.2          # weight of the D-SSIM term (Section 4.1)
PYRAMID_LEVELS = 3    # n = 2 (Section 4.1, Eq. 5)


def mapping_lr_rows(extent: float = 5.0) -> np.ndarray:
    """Per-row Adam learning rates for mapping runs that must converge.  The
    paper gives none; these follow common 3D Gaussian splatting practice:
    means 1.6e-4 x scene extent, log-scales 5e-3, quaternions 1e-3, opacity
    logit 5e-2, SH DC 2.5e-3, higher SH 1.25e-4."""
    lr = np.empty(59, np.float32)
    lr[0:3] = 1.6e-4 * extent
    lr[3:6] = 5e-3
    lr[6:10] = 1e-3
    lr[10] = 5e-2
    lr[11:14] = 2.5e-3
    lr[14:] = 1.25e-4
    return lr


class PyramidSchedule:
    """Eq. 5 coarse-to-fine supervision per keyframe (Section 3.4): a keyframe
    is first supervised at the top level n of its Gaussian pyramid and moves
    one level finer every `tau` times it is used, down to level 0.  The paper
    does not give the number of uses per level; tau = 4 is the reading taken
    here (a keyframe spends its first uses on the coarse levels)."""

    def __init__(self, levels: int = PYRAMID_LEVELS, tau: int = 4):
        if levels < 1 or tau < 1:
            raise ValueError("levels and tau must be positive")
        self.top = levels - 1
        self.tau = tau
        self.uses: dict = {}

    def level(self, keyframe) -> int:
        """Pyramid level the next use of `keyframe` is supervised at."""
        return max(0, self.top - self.uses.get(keyframe, 0) // self.tau)

    def use(self, keyframe) -> int:
        """Level for this use of `keyframe`; counts the use."""
        lv = self.level(keyframe)
        self.uses[keyframe] = self.uses.get(keyframe, 0) + 1
        return lv


def _bytes(n: int, device) -> torch.Tensor:
    return torch.empty(max(int(n), 256), dtype=torch.uint8, device=device)


def auto_bwd_waves(total_tiles: int) -> int:
    """Waves per tile for the backward raster of a plan whose settings leave
    it open (bwd_waves 0).  One wave per tile keeps the chip's 1,024 SIMDs
    busy from about 1.5 tiles per SIMD on; a plan with fewer tiles (a coarse
    pyramid level) splits each tile over two or four waves.  Measured on the
    realistic mapping workload: 1200x680 (3,225 tiles) is fastest at one
    wave, 600x340 (836) at two, 300x170 (209) at four.  Results do not depend
    on the choice."""
    if total_tiles >= 1536:
        return 1
    if total_tiles >= 512:
        return 2
    return 4


class RenderPlan:
    """Render targets = (view, pyramid level) pairs over a set of keyframe views."""

    def __init__(self, cams, specs, n_cap: int, pair_cap: int, settings=None, device="cuda",
                 tile_w: int = gs.TILE):
        self.device = torch.device(device)
        self.tile_w = int(tile_w)   # tiles of tile_w x (256 / tile_w) pixels
        self.settings = settings if settings is not None else gs.default_settings()
        self.n_cap = int(n_cap)
        self.pair_cap = int(pair_cap)
        self.cams = list(cams)
        self.views = [gs.make_view(c) for c in self.cams]
        self.n_views = len(self.views)
        self.specs = [(int(v), int(l), tuple(bg), float(w)) for (v, l, bg, w) in specs]
        self.targets, self.total_pixels, self.total_tiles = gs.gs_targets_layout(self.views, self.specs,
                                                                                 self.tile_w)
        if self.settings.bwd_waves == 0:   # left open: chosen from the plan's tile count (own copy)
            self.settings = type(self.settings).from_buffer_copy(self.settings)
            self.settings.bwd_waves = auto_bwd_waves(self.total_tiles)
        self.n_targets = len(self.specs)
        varr = (gs.gs_view * self.n_views)(*self.views)
        self.views_dev = gs.to_device_struct_array(varr, self.device)
        self.targets_dev = gs.to_device_struct_array(self.targets, self.device)
        self.sizes = gs.gs_workspace_query(self.settings, self.n_cap, self.n_views, self.targets,
                                           self.pair_cap)
        d = self.device
        self.proj_ws = _bytes(self.sizes.proj_bytes, d)
        self.sort_ws = _bytes(self.sizes.sort_bytes, d)
        self.accum_ws = _bytes(self.sizes.accum_bytes, d)
        self.loss_ws = _bytes(self.sizes.loss_bytes, d)
        P = self.total_pixels
        self.rgb = torch.empty(3 * P, dtype=torch.float32, device=d)
        self.T = torch.empty(P, dtype=torch.float32, device=d)
        self.last = torch.empty(P, dtype=torch.int32, device=d)
        self.ncontrib = torch.empty(P, dtype=torch.int32, device=d)
        self.nevals = torch.empty(P, dtype=torch.int32, device=d)
        self.status = torch.zeros(1, dtype=torch.int32, device=d)
        self.d_loss = torch.zeros(self.n_targets, dtype=torch.float32, device=d)
        self.d_total = torch.zeros(1, dtype=torch.float32, device=d)
        self.dL = torch.zeros(3 * P, dtype=torch.float32, device=d)
        # (owner, parameter version) whose projection records proj_ws holds,
        # when written by a fused optimiser step; None otherwise
        self.records_of = None

    # -- layout helpers ---------------------------------------------------
    def target_slice(self, i: int):
        t = self.targets[i]
        return int(t.pix_offset), int(t.width), int(t.height)

    def image(self, buf: torch.Tensor, i: int) -> torch.Tensor:
        """View of target i's planar [3, H, W] image inside a packed buffer."""
        off, w, h = self.target_slice(i)
        return buf[3 * off: 3 * (off + w * h)].view(3, h, w)

    def plane(self, buf: torch.Tensor, i: int) -> torch.Tensor:
        off, w, h = self.target_slice(i)
        return buf[off: off + w * h].view(h, w)

    # -- steps ----------------------------------------------------------------
    def preprocess(self, params: torch.Tensor, n: int, stream=None):
        gs.gs_preprocess(self.settings, params, n, self.views_dev, self.n_views, self.proj_ws, stream)
        self.records_of = None

    def bin_sort(self, n: int, stream=None):
        gs.gs_bin_sort(self.settings, self.proj_ws, n, self.n_cap, self.n_views, self.targets_dev,
                       self.n_targets, self.total_tiles, self.sort_ws, self.pair_cap, self.status,
                       stream)

    def render_fwd(self, with_ncontrib: bool = False, stream=None):
        gs.gs_render_fwd(self.settings, self.proj_ws, self.n_cap, self.n_views, self.sort_ws,
                         self.pair_cap, self.targets_dev, self.n_targets, self.total_tiles, self.rgb,
                         self.T, self.last, self.ncontrib if with_ncontrib else None, stream,
                         out_nevals=self.nevals if with_ncontrib else None)

    def render(self, params, n, with_ncontrib=False, stream=None):
        self.preprocess(params, n, stream)
        self.bin_sort(n, stream)
        self.render_fwd(with_ncontrib, stream)
        return self.rgb

    def loss(self, target_rgb: torch.Tensor, lam: float = LAMBDA, with_grad: bool = True, stream=None):
        gs.gs_pyramid_loss(self.rgb, target_rgb, self.targets_dev, self.n_targets, self.total_tiles,
                           self.total_pixels, lam, self.loss_ws, self.d_loss, self.d_total,
                           self.dL if with_grad else None, stream)
        return self.d_total

    def backward(self, params, n, dL_drgb, grad, stream=None):
        gs.gs_render_bwd(self.settings, params, n, self.views_dev, self.n_views, self.proj_ws,
                         self.sort_ws, self.pair_cap, self.targets_dev, self.n_targets,
                         self.total_tiles, self.T, self.last, dL_drgb, self.accum_ws, grad, stream)

    def pair_count(self) -> int:
        """Number of (tile, Gaussian) pairs of the last bin_sort (synchronises)."""
        counters = self.sort_ws[:64].view(torch.int32)
        return int(counters[1].item())

    def overflowed(self) -> bool:
        return bool(int(self.status.item()) & gs.STATUS_PAIR_OVERFLOW)


@dataclass
class Mapper:
    """Parameter store + Adam state for the mapping optimisation."""

    params: torch.Tensor
    n: int
    lr_rows: np.ndarray = field(default_factory=lambda: np.full(59, 1e-3, np.float32))
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    step_count: int = 0

    def __post_init__(self):
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.version = 0   # bumped by every change of the parameters

    def invalidate(self):
        """Call after changing the parameters outside step() (e.g. appending)."""
        self.version += 1

    def step(self, plan: RenderPlan, target_rgb: torch.Tensor, lam: float = LAMBDA, fused: bool = True,
             stream=None):
        """One iteration: render every target, Eq. 4 loss, backward, Adam.

        fused=True applies Adam inside the backward's per-Gaussian pass
        (gs_render_bwd_adam), which also writes the projection records of the
        updated parameters into the plan, so the next step on the same plan
        skips gs_preprocess; fused=False runs gs_render_bwd into a zeroed
        gradient and then gs_adam_step."""
        if not (fused and plan.records_of == (id(self), self.version)):
            plan.preprocess(self.params, self.n, stream)
        plan.bin_sort(self.n, stream)
        plan.render_fwd(stream=stream)
        plan.loss(target_rgb, lam, True, stream)
        self.step_count += 1
        self.version += 1
        if fused:
            gs.gs_render_bwd_adam(plan.settings, self.params, self.n, plan.views_dev, plan.n_views,
                                  plan.proj_ws, plan.sort_ws, plan.pair_cap, plan.targets_dev,
                                  plan.n_targets, plan.total_tiles, plan.T, plan.last, plan.dL,
                                  plan.accum_ws, self.m, self.v, self.lr_rows, self.step_count,
                                  self.beta1, self.beta2, self.eps, plan.proj_ws, stream)
            plan.records_of = (id(self), self.version)
        else:
            gs.gs_fill(self.grad, 0.0, stream)
            plan.backward(self.params, self.n, plan.dL, self.grad, stream)
            gs.gs_adam_step(self.params, self.grad, self.m, self.v, self.n, self.lr_rows,
                            self.step_count, self.beta1, self.beta2, self.eps, stream)
        return plan.d_total
