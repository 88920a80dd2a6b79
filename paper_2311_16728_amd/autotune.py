"""Autotuner for the rasteriser's launch shape.

Candidates: tile shape (tile_w x 256/tile_w pixels, tile_w 8, 16, 32; one
render plan per shape, built by the caller's factory) x forward LDS batch
(64, 128, 256 Gaussians staged per round) x backward waves per tile (1, 2, 4;
i.e. 4, 2, 1 pixels per lane); the best of those is then also timed with the
persistent raster launch over the cost-ordered tile queue (schedule 1: forward
and backward; 2: backward only) and keeps the fastest.  Each candidate runs whole mapping iterations
(preprocess, sort, forward, loss, backward, Adam on a scratch copy of the
parameters), timed with HIP events on the launch stream; the fastest is kept.
The forward image does not depend on the choice (inclusion is per pixel and
the list order is fixed), which the tuner checks bitwise across every
candidate.  Choices are cached per (device, shape class).
"""

from __future__ import annotations

import itertools
import json
import os

import torch

from . import gs

BATCHES = (64, 128, 256)
BWD_WAVES = (1, 2, 4)
TILE_WIDTHS = (8, 16, 32)
_cache: dict = {}


def shape_class(plan, n: int) -> str:
    """Bucket of the problem: Gaussians and pixels to the nearest power of two, targets."""
    def b2(x):
        return 1 << max(0, int(x) - 1).bit_length()
    return f"n{b2(n)}-px{b2(plan.total_pixels)}-t{plan.n_targets}"


def _key(plan, n):
    dev = torch.cuda.get_device_name(plan.device)
    return f"{dev}|{shape_class(plan, n)}|w{plan.tile_w}"


def load(path: str):
    if path and os.path.exists(path):
        with open(path) as f:
            _cache.update(json.load(f))


def save(path: str):
    if path:
        with open(path, "w") as f:
            json.dump(_cache, f, indent=1, sort_keys=True)


def tune(plan, params: torch.Tensor, n: int, target: torch.Tensor, iters: int = 5, warmup: int = 2,
         path: str | None = None, force: bool = False, ref_img: torch.Tensor | None = None):
    """Pick (batch, bwd_waves) for `plan` (its tile shape fixed); sets
    plan.settings and returns the choice with the measured ms per iteration
    of every candidate.  Every candidate's forward image must equal the first
    one bitwise; ref_img (from another tile shape) must be matched to within
    1e-2 (the staged offsets' FP32 rounding depends on the tile origin, so a
    near-cutoff decision can flip, moving a pixel by about alpha_min)."""
    load(path)
    key = _key(plan, n)
    if key in _cache and not force:
        c = _cache[key]
        plan.settings.batch, plan.settings.bwd_waves = c["batch"], c["bwd_waves"]
        plan.settings.schedule = c.get("schedule", 0)
        return c
    p = params.detach().clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    lr = [1e-4] * gs.NUM_ROWS
    timings = {}
    other, ref_img = ref_img, None

    def run(label):
        nonlocal ref_img
        plan.render(params, n)
        torch.cuda.synchronize()
        img = plan.rgb.clone()
        if other is not None and float((img - other).abs().max()) > 1e-2:
            raise RuntimeError(f"forward of tile_w={plan.tile_w} differs from another tile shape")
        if ref_img is None:
            ref_img = img
        elif not torch.equal(img, ref_img):
            raise RuntimeError(f"forward differs for tile_w={plan.tile_w} {label}: "
                               "results must not depend on the launch shape")
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
        timings[label] = e0.elapsed_time(e1) / iters

    plan.settings.schedule = 0
    for batch, waves in itertools.product(BATCHES, BWD_WAVES):
        plan.settings.batch, plan.settings.bwd_waves = batch, waves
        run(f"{batch}x{waves}")
    best = min(timings, key=timings.get)
    b, w = (int(x) for x in best.split("x"))
    plan.settings.batch, plan.settings.bwd_waves = b, w
    # the same launch shape over the cost-ordered tile queue: forward and
    # backward (1), backward only (2)
    label = {0: best, 1: f"{b}x{w}q", 2: f"{b}x{w}qb"}
    for sched in (1, 2):
        plan.settings.schedule = sched
        run(label[sched])
    sched = min((0, 1, 2), key=lambda k: timings[label[k]])
    plan.settings.schedule = sched
    _cache[key] = {"batch": b, "bwd_waves": w, "schedule": sched, "ms": timings}
    save(path)
    return _cache[key]


def tune_tiles(make_plan, params: torch.Tensor, n: int, target: torch.Tensor,
               tile_ws=TILE_WIDTHS, iters: int = 5, warmup: int = 2, path: str | None = None):
    """Tile shape as well: make_plan(tile_w) builds a render plan for each
    candidate width; each is tuned with `tune`, the forward images of all
    candidates must agree bitwise.  Returns (plan, choice) for the fastest;
    the other plans are released."""
    best_plan, best, per_shape, ref_img = None, None, {}, None
    for tw in tile_ws:
        plan = make_plan(tw)
        c = tune(plan, params, n, target, iters, warmup, path, force=True, ref_img=ref_img)
        if ref_img is None:
            plan.render(params, n)
            torch.cuda.synchronize()
            ref_img = plan.rgb.clone()
        ms = c["ms"][f"{c['batch']}x{c['bwd_waves']}" + ("", "q", "qb")[c["schedule"]]]
        per_shape[tw] = c["ms"]
        if best is None or ms < best["best_ms"]:
            if best_plan is not None:
                del best_plan
                torch.cuda.empty_cache()
            best_plan = plan
            best = {"tile_w": tw, "batch": c["batch"], "bwd_waves": c["bwd_waves"], "schedule": c["schedule"],
                    "best_ms": ms}
        else:
            del plan
            torch.cuda.empty_cache()
    best["ms"] = per_shape
    return best_plan, best
