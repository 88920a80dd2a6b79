"""Online photorealistic mapping with per-keyframe Gaussian-pyramid levels.

Keyframes join the mapper over time (Section 3.3).  Every iteration trains
one keyframe, picked uniformly among those that have joined, at the pyramid
level its own use count selects (Section 3.4, Eq. 5: level n first, one level
finer every `tau` uses, then level 0), then steps Adam; gradient-driven
densification runs every `densify_every` iterations, and a joining keyframe
can bring new primitives at its inactive keypoints (geometry-based
densification, Section 3.3.1).  One render plan per pyramid level holds the
workspaces; the keyframe's pose is written into the plan's view slot before
its iteration, so any number of keyframes costs no extra device memory
beyond their ground-truth pyramids.

``online_scene`` builds the synthetic stand-in: a seeded room map as the
ground truth, its renders at keyframes on a random walk, a sparse initial map
(a fraction of the ground-truth centres, optionally jittered as a monocular
depth error would, with heuristic shape and colour), and per keyframe the
held-out ground-truth centres visible in it as keypoints.
"""

from __future__ import annotations

import math
import time

import numpy as np
import torch

import scenes
from . import gs
from .densify import Densifier
from .mapper import LAMBDA, Mapper, PyramidSchedule, RenderPlan, mapping_lr_rows


class OnlineMapper:
    def __init__(self, params: torch.Tensor, n: int, cams, gt_images, levels: int = 3, tau: int = 4,
                 lr_rows=None, pair_cap: int = 1 << 26, settings=None, densify_every: int = 0,
                 extent: float = 5.0, seed: int = 0):
        dev = params.device
        if len({(c["width"], c["height"]) for c in cams}) != 1:
            raise ValueError("keyframes must share one image size (one plan per level serves them all)")
        self.mapper = Mapper(params, n, lr_rows=mapping_lr_rows(extent) if lr_rows is None else lr_rows)
        self.cams = list(cams)
        self.levels = levels
        self.schedule = PyramidSchedule(levels, tau)
        n_cap = params.shape[1]
        if settings is None:   # the backward's waves per tile chosen per level (auto_bwd_waves)
            settings = gs.default_settings(bwd_waves=0)
        self.plans = [RenderPlan([self.cams[0]], [(0, l, (0.0, 0.0, 0.0), 1.0)], n_cap, pair_cap, settings, dev)
                      for l in range(levels)]
        self.view_dev = [gs.to_device_struct_array((gs.gs_view * 1)(gs.make_view(c)), dev) for c in self.cams]
        # ground-truth pyramid of every keyframe, level by level
        self.gt = []
        for img in gt_images:
            H, W = img.shape[1], img.shape[2]
            sizes = []
            h, w = H, W
            for _ in range(levels):
                sizes.append(3 * h * w)
                h, w = (h + 1) // 2, (w + 1) // 2
            pyr = torch.empty(sum(sizes), dtype=torch.float32, device=dev)
            gs.gs_pyramid_build(img.contiguous(), levels, pyr)
            self.gt.append(list(torch.split(pyr, sizes)))
        self.active: list[int] = []
        self.rng = np.random.default_rng(seed)
        self.densify_every = densify_every
        self.densifier = Densifier(self.mapper, extent) if densify_every else None
        self.iteration = 0
        self.log: list[tuple[int, int]] = []     # (keyframe, level) per iteration

    def bind(self, level: int, k: int) -> RenderPlan:
        """The level's plan, set up to render keyframe k."""
        plan = self.plans[level]
        plan.views_dev.copy_(self.view_dev[k])
        plan.cams = [self.cams[k]]
        plan.records_of = None
        return plan

    def add_keyframe(self, k: int, new_params: torch.Tensor | None = None):
        """Keyframe k joins; new_params ([59][B], device) are appended."""
        self.active.append(k)
        if new_params is not None and new_params.shape[1] > 0:
            mp = self.mapper
            gs.gs_append(mp.params, mp.m, mp.v, mp.n, new_params)
            mp.n += new_params.shape[1]
            mp.invalidate()

    def step(self):
        k = self.active[int(self.rng.integers(len(self.active)))]
        level = self.schedule.use(k)
        plan = self.bind(level, k)
        self.mapper.step(plan, self.gt[k][level], LAMBDA)
        self.iteration += 1
        self.log.append((k, level))
        if self.densifier is not None:
            self.densifier.accumulate(plan)
            if self.iteration % self.densify_every == 0:
                self.densifier.densify()

    def psnr(self, keyframes=None) -> float:
        """Mean level-0 PSNR over keyframes (all joined ones by default)."""
        vals = []
        for k in (self.active if keyframes is None else keyframes):
            plan = self.bind(0, k)
            plan.render(self.mapper.params, self.mapper.n)
            a = plan.rgb.clamp(0, 1)
            b = self.gt[k][0].clamp(0, 1)
            vals.append(10.0 * math.log10(1.0 / max(float(((a - b) ** 2).mean()), 1e-12)))
        return float(np.mean(vals))

    def render_fps(self, keyframes, reps: int = 3) -> float:
        """Level-0 rendering rate (projection + binning + forward) over keyframes."""
        plan = self.plans[0]
        for k in keyframes:
            self.bind(0, k)
            plan.render(self.mapper.params, self.mapper.n)
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(reps):
            for k in keyframes:
                self.bind(0, k)
                plan.render(self.mapper.params, self.mapper.n)
        t1.record()
        torch.cuda.synchronize()
        return 1000.0 * reps * len(keyframes) / t0.elapsed_time(t1)


def _visible_weight(Pgt, n, cam, n_cap, device):
    """Per ground-truth Gaussian, its summed alpha * T over the keyframe's
    pixels (the colour-DC gradient of an all-ones loss divided by Y_0)."""
    one = RenderPlan([cam], [(0, 0, (0, 0, 0), 1.0)], n_cap, 1 << 26, None, device)
    one.render(Pgt, n)
    dL = torch.zeros(3 * one.total_pixels, dtype=torch.float32, device=device)
    dL[:one.total_pixels] = 1.0
    grad = torch.zeros_like(Pgt)
    one.backward(Pgt, n, dL, grad)
    if one.overflowed():
        raise RuntimeError("pair buffer overflow while scoring visibility")
    return (grad[11, :n] / 0.28209479177387814).cpu().numpy()


def _project(cam, mu):
    R = np.asarray(cam["R"], np.float64)
    xc = mu.T.astype(np.float64) @ R.T + np.asarray(cam["t"], np.float64)
    z = xc[:, 2]
    u = cam["fx"] * xc[:, 0] / np.maximum(z, 1e-9) + cam["cx"]
    v = cam["fy"] * xc[:, 1] / np.maximum(z, 1e-9) + cam["cy"]
    return u, v, z


def online_scene(seed: int, n_gt: int = 300_000, n_kf: int = 16, width: int = 1200, height: int = 680,
                 f: float = 600.0, init_frac: float = 0.15, pos_noise: float = 0.0, per_kf: int = 2000,
                 n_cap: int | None = None, device="cuda") -> dict:
    """The synthetic online-mapping workload (see the module docstring)."""
    gt, _, cams = scenes.room_scene(seed, n_gt, n_kf, width, height, f)
    rng = np.random.default_rng(seed + 7)
    Pgt = torch.as_tensor(gt).to(device)
    ref = RenderPlan(cams, [(v, 0, (0, 0, 0), 1.0) for v in range(n_kf)], gt.shape[1], 1 << 28, None, device)
    ref.render(Pgt, n_gt)
    if ref.overflowed():
        raise RuntimeError("pair buffer overflow while rendering the ground truth")
    gt_images = [ref.image(ref.rgb, v).clone() for v in range(n_kf)]
    del ref
    # held-out keypoints per keyframe: visible ground-truth centres not in the initial map
    init = rng.uniform(size=n_gt) < init_frac
    taken = init.copy()
    kps = []
    for k, cam in enumerate(cams):
        w = _visible_weight(Pgt, n_gt, cam, gt.shape[1], device)
        u, v, z = _project(cam, gt[0:3, :n_gt])
        ok = (w >= 1.0) & (z > 0.3) & (u >= 0) & (u < width - 1) & (v >= 0) & (v < height - 1) & ~taken
        cand = np.nonzero(ok)[0]
        pick = np.sort(rng.choice(cand, size=min(per_kf, cand.size), replace=False))
        taken[pick] = True
        kps.append(pick)
    # colour of a centre: the ground-truth image at its projection in the
    # first keyframe that sees it in front (grey if none)
    def colours(idx):
        rgb = np.full((3, idx.size), 0.5, np.float32)
        done = np.zeros(idx.size, bool)
        for k, cam in enumerate(cams):
            u, v, z = _project(cam, gt[0:3, idx])
            ok = ~done & (z > 0.3) & (u >= 0) & (u <= width - 1) & (v >= 0) & (v <= height - 1)
            if ok.any():
                img = gt_images[k].cpu().numpy()
                rgb[:, ok] = img[:, np.rint(v[ok]).astype(int), np.rint(u[ok]).astype(int)]
                done |= ok
        return rgb
    init_idx = np.nonzero(init)[0]
    mu0 = gt[0:3, init_idx] + rng.normal(0.0, pos_noise, size=(3, init_idx.size)).astype(np.float32)
    total = init_idx.size + sum(len(p) for p in kps)
    n_cap = n_cap or scenes.pad_cap(8 * total)   # room for gradient-driven densification
    P = torch.zeros(59, n_cap, dtype=torch.float32, device=device)
    heur = torch.empty(59, init_idx.size, dtype=torch.float32, device=device)
    gs.gs_init_heuristic(torch.as_tensor(mu0).to(device).contiguous(),
                         torch.as_tensor(colours(init_idx)).to(device).contiguous(), P, 0, heur)
    gs.gs_append(P, None, None, 0, heur)
    new_mu, new_rgb = [], []
    for pick in kps:
        mu = gt[0:3, pick] + rng.normal(0.0, pos_noise, size=(3, pick.size)).astype(np.float32)
        new_mu.append(torch.as_tensor(mu).to(device).contiguous())
        new_rgb.append(torch.as_tensor(colours(pick)).to(device).contiguous())
    return dict(cams=cams, gt_images=gt_images, params=P, n=int(init_idx.size), new_mu=new_mu,
                new_rgb=new_rgb, n_gt=n_gt)


def run_online(sc: dict, levels: int, tau: int = 4, geo: bool = True, iters: int = 2400,
               join_every: int = 100, densify_every: int = 100, seed: int = 0, settings=None) -> dict:
    """One online run over a scene from online_scene: keyframe k joins at
    iteration k * join_every (with its keypoints' primitives when geo)."""
    P = sc["params"].clone()
    om = OnlineMapper(P, sc["n"], sc["cams"], sc["gt_images"], levels=levels, tau=tau,
                      densify_every=densify_every, seed=seed, settings=settings)
    n_kf = len(sc["cams"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        if it % join_every == 0 and it // join_every < n_kf:
            k = it // join_every
            new = None
            B = sc["new_mu"][k].shape[1]
            if geo and B > 0:
                mp = om.mapper
                new = torch.empty(59, B, dtype=torch.float32, device=P.device)
                gs.gs_init_heuristic(sc["new_mu"][k], sc["new_rgb"][k], mp.params, mp.n, new)
            om.add_keyframe(k, new)
        om.step()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    for p in om.plans:
        if p.overflowed():
            raise RuntimeError("pair buffer overflow during the online run")
    return dict(levels=levels, geo=geo, iters=iters, seconds=round(secs, 3),
                iters_per_s=round(iters / secs, 1), psnr=round(om.psnr(list(range(n_kf))), 3),
                fps=round(om.render_fps(list(range(n_kf))), 1), primitives=om.mapper.n,
                mb=round(om.mapper.n * 59 * 4 / 1e6, 3), mapper=om)
