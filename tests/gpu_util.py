"""Helpers shared by the GPU tests: build render plans, read workspaces back."""

from __future__ import annotations

import numpy as np
import torch

import scenes


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm device (torch.cuda.is_available() is False)")
    from paper_2311_16728_amd import gs  # noqa: F401  (fails loudly without libgs.so)


def plan_for(cams, levels=(0,), bgs=None, n_cap=256, pair_cap=1 << 20, settings=None, weights=None,
             tile_w=16):
    from paper_2311_16728_amd.mapper import RenderPlan

    specs = []
    for vi, _ in enumerate(cams):
        for l in levels:
            bg = tuple(np.asarray(cams[vi].get("bg", (0, 0, 0)), np.float64)) if bgs is None else bgs
            w = 1.0 if weights is None else weights[len(specs)]
            specs.append((vi, l, bg, w))
    return RenderPlan(cams, specs, n_cap, pair_cap, settings, tile_w=tile_w)


def proj_records(plan, n):
    """(mean [R,2], cov_o [R,4], rgb_z [R,4]) as numpy, R = n_views * n_cap."""
    R = plan.n_views * plan.n_cap

    def up(x):
        return (x + 255) // 256 * 256

    ws = plan.proj_ws
    o_mean, o_cov = 0, up(16 * R)
    o_rgb = o_cov + up(16 * R)
    mean = ws[o_mean:o_mean + 16 * R].view(torch.float64).view(R, 2).cpu().numpy()
    cov = ws[o_cov:o_cov + 16 * R].view(torch.float32).view(R, 4).cpu().numpy()
    rgb = ws[o_rgb:o_rgb + 16 * R].view(torch.float32).view(R, 4).cpu().numpy()
    return mean, cov, rgb


def level_cam(cam, level):
    return scenes.level_camera(cam, level) if level else cam


def compare_image(gpu_img, gpu_T, orc, tol=1e-4):
    """max |diff| over non-ambiguous pixels; returns (max_img, max_T, n_amb)."""
    from oracle import AMB_IMAGE

    ok = (orc["amb"] & AMB_IMAGE) == 0
    d_img = np.abs(gpu_img - orc["img"]).max(axis=0)
    d_T = np.abs(gpu_T - orc["T"])
    return float(d_img[ok].max()), float(d_T[ok].max()), int((~ok).sum()), d_img, ok


def group_rel_err(g, ref, ids):
    """Per (Gaussian, group) relative error with the floor of the gradient metric:
    ||g - ref|| / max(||ref||, 1e-3 * median ||ref|| over the chosen Gaussians)."""
    groups = {"mean": slice(0, 3), "logscale": slice(3, 6), "quat": slice(6, 10),
              "opacity": slice(10, 11), "sh": slice(11, 59)}
    out = {}
    for name, sl in groups.items():
        r = ref[sl][:, ids]
        d = g[sl][:, ids] - r
        nr = np.linalg.norm(r, axis=0)
        floor = 1e-3 * np.median(nr)
        out[name] = np.linalg.norm(d, axis=0) / np.maximum(nr, max(floor, 1e-30))
    return out


def check_gradients(g, ref, candidates, label="", n_sample=64, tol=1e-3, seed=0, p99=0.1):
    """The gradient metric: 64 Gaussians drawn with `seed` from `candidates`
    (Gaussians with a composited pixel) must have relative error <= tol in every
    group; over all candidates the 99th percentile must stay <= p99 * tol and the
    worst case <= 5 tol (scalar groups such as the opacity can cancel over
    random-sign pixel weights, which amplifies FP32 rounding of single terms)."""
    candidates = np.asarray(candidates)
    rng = np.random.default_rng(seed)
    ids = rng.choice(candidates, min(n_sample, len(candidates)), replace=False)
    sampled = group_rel_err(g, ref, ids)
    every = group_rel_err(g, ref, candidates)
    for k in sampled:
        print(f"{label} {k}: sampled max {sampled[k].max():.2e}; all p99 {np.quantile(every[k], 0.99):.2e} "
              f"max {every[k].max():.2e}")
    for k in sampled:
        assert sampled[k].max() <= tol, (k, float(sampled[k].max()))
        assert np.quantile(every[k], 0.99) <= p99 * tol, k
        assert every[k].max() <= 5 * tol, k
