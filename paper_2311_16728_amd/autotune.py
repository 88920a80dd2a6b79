"""Autotuner for the rasteriser's launch shape.

Candidates: forward LDS batch (64, 128, 256 Gaussians staged per round) x
backward waves per 16x16 tile (1, 2, 4; i.e. 4, 2, 1 pixels per lane).  Each
candidate runs whole mapping iterations on the caller's plan (preprocess, sort,
forward, loss, backward, Adam on a scratch copy of the parameters), timed with
HIP events on the launch stream; the fastest is kept.  The forward result does
not depend on the choice (inclusion is per pixel and the list order is fixed),
which `tune` checks bitwise.  Choices are cached per (device, shape class).
"""

from __future__ import annotations

import itertools
import json
import os

import torch

from . import gs

BATCHES = (64, 128, 256)
BWD_WAVES = (1, 2, 4)
_cache: dict = {}


def shape_class(plan, n: int) -> str:
    """Bucket of the problem: Gaussians and pixels to the nearest power of two, targets."""
    def b2(x):
        return 1 << max(0, int(x) - 1).bit_length()
    return f"n{b2(n)}-px{b2(plan.total_pixels)}-t{plan.n_targets}"


def _key(plan, n):
    dev = torch.cuda.get_device_name(plan.device)
    return f"{dev}|{shape_class(plan, n)}"


def load(path: str):
    if path and os.path.exists(path):
        with open(path) as f:
            _cache.update(json.load(f))


def save(path: str):
    if path:
        with open(path, "w") as f:
            json.dump(_cache, f, indent=1, sort_keys=True)


def tune(plan, params: torch.Tensor, n: int, target: torch.Tensor, iters: int = 5, warmup: int = 2,
         path: str | None = None, force: bool = False):
    """Pick (batch, bwd_waves) for `plan`; sets plan.settings and returns the choice
    with the measured ms per iteration of every candidate."""
    load(path)
    key = _key(plan, n)
    if key in _cache and not force:
        c = _cache[key]
        plan.settings.batch, plan.settings.bwd_waves = c["batch"], c["bwd_waves"]
        return c
    base = (plan.settings.batch, plan.settings.bwd_waves)
    p = params.detach().clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    lr = [1e-4] * gs.NUM_ROWS
    ref_img = None
    timings = {}
    for batch, waves in itertools.product(BATCHES, BWD_WAVES):
        plan.settings.batch, plan.settings.bwd_waves = batch, waves
        plan.render(params, n)
        torch.cuda.synchronize()
        img = plan.rgb.clone()
        if ref_img is None:
            ref_img = img
        elif not torch.equal(img, ref_img):
            raise RuntimeError(f"forward differs for batch={batch}: results must not depend on it")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        step = 0
        for it in range(warmup + iters):
            if it == warmup:
                e0.record()
            plan.render(p, n)
            plan.loss(target)
            step += 1
            gs.gs_render_bwd_adam(plan.settings, p, n, plan.views_dev, plan.n_views, plan.proj_ws,
                                  plan.sort_ws, plan.pair_cap, plan.targets_dev, plan.n_targets,
                                  plan.total_tiles, plan.T, plan.last, plan.dL, plan.accum_ws, m, v,
                                  lr, step)
        e1.record()
        torch.cuda.synchronize()
        timings[f"{batch}x{waves}"] = e0.elapsed_time(e1) / iters
    best = min(timings, key=timings.get)
    b, w = (int(x) for x in best.split("x"))
    plan.settings.batch, plan.settings.bwd_waves = b, w
    _cache[key] = {"batch": b, "bwd_waves": w, "ms": timings}
    save(path)
    del base
    return _cache[key]
