"""A scene built so that float32 and FP64 take different compositing decisions
(Section 3.3, Eq. 3) at many pixels: the input that gives the FP32-ambiguity
classifier's pin its teeth, and a parity case for the GPU.

Four groups of primitives in front of a tilted 64x64 camera:

* clutter: ordinary primitives (the tiny workload's laws);
* cutoff pins: each primitive's opacity is set so that at one chosen pixel
  its opacity o * exp(power) equals 1/255 up to the float32 rounding of the
  opacity logit (|ln(255 o e^power)| ~ 1e-7);
* stop pins: pairs of opaque primitives (logit 14, so the 0.99 clamp) on one
  pixel centre at two depths: the transmittance after both is (1 - 0.99)^2,
  just above 1e-4 in FP64 and just below it in float32;
* depth pins: a primitive and a copy whose mean is moved by a few float32
  ulp so that its FP64 depth is smaller by less than a float32 ulp of the
  depth; both round to the same float32 depth (then index order) while FP64
  puts the copy first.  The copy has another colour.

Built from the oracle's own projection records (the opacity and position
choices need the projected covariance and depth); nothing here comes from the
GPU path.
"""

from __future__ import annotations

import numpy as np

import scenes

ALPHA_MIN = 1.0 / 255.0


def _rot(axis, angle):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)


def camera():
    return scenes.pinhole(64, 64, 64.0, 64.0, 32.0, 32.0, R=_rot([0.3, 1.0, 0.2], 0.07),
                          t=[0.05, -0.02, 0.1], bg=(0.1, 0.2, 0.3))


def _world(cam, u, v, z):
    """World point seen at pixel (u, v) at camera depth z."""
    R = np.asarray(cam["R"], np.float64)
    t = np.asarray(cam["t"], np.float64)
    xc = np.stack([(u - cam["cx"]) / cam["fx"] * z, (v - cam["cy"]) / cam["fy"] * z, z])
    return (R.T @ (xc - t[:, None])).astype(np.float32)


def _depth64(cam, mu):
    R = np.asarray(cam["R"], np.float64)
    t = np.asarray(cam["t"], np.float64)
    mu = np.asarray(mu, np.float64)
    return R[2, 0] * mu[0] + R[2, 1] * mu[1] + R[2, 2] * mu[2] + t[2]


def knife_edge_scene(orc, seed: int = 0):
    """Returns (params, n, cam, groups): groups[k] = column indices of group k."""
    rng = np.random.default_rng(seed)
    cam = camera()
    W, H = cam["width"], cam["height"]
    n_bg, n_cut, n_stack, n_tie = 300, 160, 12, 24
    n = n_bg + n_cut + 2 * n_stack + 2 * n_tie
    p = np.zeros((59, scenes.pad_cap(n)), np.float32)
    base = scenes.draw_gaussians(rng, n, (0, 0, 0), (1, 1, 1))[:, :n]
    p[:, :n] = base
    cols = np.arange(n)
    g_bg = cols[:n_bg]
    g_cut = cols[n_bg:n_bg + n_cut]
    g_stack = cols[n_bg + n_cut:n_bg + n_cut + 2 * n_stack]
    g_tie = cols[n_bg + n_cut + 2 * n_stack:]

    # clutter and cutoff pins: random pixels and depths
    m = n_bg + n_cut
    p[0:3, :m] = _world(cam, rng.uniform(-4, W + 4, m), rng.uniform(-4, H + 4, m),
                        rng.uniform(2.0, 4.0, m))
    p[3:6, n_bg:m] = rng.normal(-3.0, 0.3, (3, n_cut))
    p[10, n_bg:m] = 0.0

    # stop pins: two opaque primitives centred on one pixel centre
    us = rng.integers(6, W - 6, n_stack).astype(np.float64)
    vs = rng.integers(6, H - 6, n_stack).astype(np.float64)
    front, back = g_stack[0::2], g_stack[1::2]
    p[0:3, front] = _world(cam, us, vs, rng.uniform(1.2, 1.5, n_stack))
    p[0:3, back] = _world(cam, us, vs, rng.uniform(1.7, 1.9, n_stack))
    p[3:6, g_stack] = np.log(0.02)
    p[6:10, g_stack] = [[1.0], [0.0], [0.0], [0.0]]
    p[10, g_stack] = 14.0
    p[11:14, front] = [[1.5], [-1.0], [0.2]]
    p[11:14, back] = [[-1.0], [1.5], [0.4]]
    p[14:59, g_stack] = 0.0

    # depth pins: a primitive and a copy a few ulp away with a smaller FP64 depth
    first, second = g_tie[0::2], g_tie[1::2]
    p[0:3, first] = _world(cam, rng.uniform(8, W - 8, n_tie), rng.uniform(8, H - 8, n_tie),
                           rng.uniform(2.0, 3.0, n_tie))
    p[3:6, first] = rng.normal(-2.8, 0.2, (3, n_tie))
    p[10, g_tie] = 1.0
    for i, j in zip(first, second):
        p[:, j] = p[:, i]
        p[11:14, j] = p[11:14, i] + np.float32(1.2)
        z0 = _depth64(cam, p[0:3, i])
        found = False
        for axis in (0, 1, 2):
            x = p[axis, i]
            for k in range(1, 6):
                for sgn in (1, -1):
                    y = x
                    for _ in range(k):
                        y = np.nextafter(y, np.float32(sgn * np.inf))
                    mu = p[0:3, i].copy()
                    mu[axis] = y
                    z1 = _depth64(cam, mu)
                    if z1 < z0 and np.float32(z1) == np.float32(z0):
                        p[0:3, j] = mu
                        found = True
                        break
                if found:
                    break
            if found:
                break
        assert found, "no depth pin position found"

    # cutoff pins: opacity from the projected covariance at a chosen pixel
    f = {k: i for i, k in enumerate(orc.REC_FIELDS)}
    rec = orc.preprocess(p, n, cam)
    lo, hi = np.log(ALPHA_MIN / 0.95), np.log(ALPHA_MIN / 0.2)   # power range for o in [0.2, 0.95]
    keep = []
    for g in g_cut:
        r = rec[g]
        if r[f["valid"]] == 0:
            continue
        mx, my = r[f["mx"]], r[f["my"]]
        a, b, c = r[f["ca"]], r[f["cb"]], r[f["cc"]]
        want = rng.uniform(lo, hi)
        best = None
        for py in range(int(np.floor(my)) - 8, int(np.floor(my)) + 9):
            for px in range(int(np.floor(mx)) - 8, int(np.floor(mx)) + 9):
                if not (0 <= px < W and 0 <= py < H):
                    continue
                dx, dy = mx - px, my - py
                pw = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
                if lo <= pw <= hi and (best is None or abs(pw - want) < abs(best - want)):
                    best = pw
        if best is None:
            continue
        o = ALPHA_MIN * np.exp(-best)
        p[10, g] = np.float32(np.log(o / (1.0 - o)))
        keep.append(g)
    groups = dict(clutter=g_bg, cutoff=np.asarray(keep), stop=g_stack, depth=g_tie)
    return p, n, cam, groups
