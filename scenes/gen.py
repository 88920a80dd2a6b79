"""Seeded scene, camera and image generators (inputs only, no method arithmetic)."""

from __future__ import annotations

import math

import numpy as np

NROWS = 59
ROW_MU, ROW_LOGS, ROW_QUAT, ROW_OPAC, ROW_SH = 0, 3, 6, 10, 11


def pad_cap(n: int, align: int = 256) -> int:
    """Column capacity of the parameter store: ``n`` rounded up to ``align``."""
    return max(align, (n + align - 1) // align * align)


def draw_gaussians(rng: np.random.Generator, n: int, lo, hi, n_cap: int | None = None) -> np.ndarray:
    """Draw ``n`` Gaussians with means uniform in the box ``[lo, hi]``.

    log-scale ~ N(-3.5, 0.5) per axis; quaternion uniform on the unit sphere;
    opacity logit ~ N(0, 1); SH-DC ~ N(0.5, 0.2); other SH ~ N(0, 0.05).
    """
    n_cap = pad_cap(n) if n_cap is None else n_cap
    assert n_cap >= n
    p = np.zeros((NROWS, n_cap), np.float32)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    mu = rng.uniform(lo, hi, size=(n, 3))
    logs = rng.normal(-3.5, 0.5, size=(n, 3))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = rng.normal(0.0, 1.0, size=n)
    dc = rng.normal(0.5, 0.2, size=(n, 3))
    rest = rng.normal(0.0, 0.05, size=(n, 45))
    p[0:3, :n] = mu.T
    p[3:6, :n] = logs.T
    p[6:10, :n] = q.T
    p[10, :n] = op
    p[11:14, :n] = dc.T
    p[14:59, :n] = rest.T
    return p


def perturb(rng: np.random.Generator, params: np.ndarray, n: int, sigma: float = 0.05) -> np.ndarray:
    """Copy of ``params`` with every raw value of the first ``n`` columns perturbed by N(0, sigma)."""
    out = params.copy()
    out[:, :n] += rng.normal(0.0, sigma, size=(NROWS, n)).astype(np.float32)
    return out


def pinhole(width: int, height: int, fx: float, fy: float | None = None, cx: float | None = None,
            cy: float | None = None, R=None, t=None, bg=(0.0, 0.0, 0.0)) -> dict:
    fy = fx if fy is None else fy
    cx = width / 2.0 if cx is None else cx
    cy = height / 2.0 if cy is None else cy
    R = np.eye(3) if R is None else np.asarray(R, np.float64)
    t = np.zeros(3) if t is None else np.asarray(t, np.float64)
    f32 = lambda x: float(np.float32(x))   # both consumers see the same float32 values
    return dict(R=R.astype(np.float32), t=t.astype(np.float32), fx=f32(fx), fy=f32(fy),
                cx=f32(cx), cy=f32(cy), width=int(width), height=int(height),
                bg=np.asarray(bg, np.float32))


def level_camera(cam: dict, level: int) -> dict:
    """Camera of pyramid level ``level``: intrinsics divided by 2**level, sizes ceil-halved."""
    out = dict(cam)
    w, h = cam["width"], cam["height"]
    for _ in range(level):
        w, h = (w + 1) // 2, (h + 1) // 2
    s = 0.5 ** level
    out.update(fx=cam["fx"] * s, fy=cam["fy"] * s, cx=cam["cx"] * s, cy=cam["cy"] * s,
               width=w, height=h, level=level,
               tan_half_fov_x=0.5 * cam["width"] / cam["fx"],
               tan_half_fov_y=0.5 * cam["height"] / cam["fy"])
    return out


def _rodrigues(axis_angle: np.ndarray) -> np.ndarray:
    th = float(np.linalg.norm(axis_angle))
    if th == 0.0:
        return np.eye(3)
    k = axis_angle / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(th) * K + (1 - math.cos(th)) * (K @ K)


def random_walk(rng: np.random.Generator, n_steps: int, room_lo, room_hi, step_m: float = 0.1,
                step_deg: float = 5.0, margin: float = 1.0):
    """Smooth random walk of camera poses inside a room.

    Returns a list of (R_world_to_cam, t) pairs.  The first pose sits at the room
    centre looking along +z; each step moves 0.1 m in a random direction and
    rotates by 5 degrees about a random axis in the camera frame; positions are
    reflected to stay ``margin`` inside the room.
    """
    lo = np.asarray(room_lo, np.float64) + margin
    hi = np.asarray(room_hi, np.float64) - margin
    Rcw = np.eye(3)
    C = (np.asarray(room_lo, np.float64) + np.asarray(room_hi, np.float64)) / 2.0
    poses = []
    for i in range(n_steps):
        if i > 0:
            d = rng.normal(size=3)
            C = C + step_m * d / np.linalg.norm(d)
            C = np.where(C < lo, 2 * lo - C, C)
            C = np.where(C > hi, 2 * hi - C, C)
            a = rng.normal(size=3)
            Rcw = Rcw @ _rodrigues(math.radians(step_deg) * a / np.linalg.norm(a))
        R = Rcw.T
        poses.append((R, -R @ C))
    return poses


def tiny_scene(seed: int = 0, n: int = 2000):
    """The small workload: N Gaussians in front of one 128x128 pinhole camera (f=128, c=64).

    Returns (params, target_params, cam).  The target parameters are the raw
    parameters perturbed by N(0, 0.05); the caller renders them to get the
    target image.
    """
    rng = np.random.default_rng(seed)
    p = draw_gaussians(rng, n, (-1, -1, 2), (1, 1, 4))
    tgt = perturb(rng, p, n)
    cam = pinhole(128, 128, 128.0, 128.0, 64.0, 64.0)
    return p, tgt, cam


ROOM_LO = (-5.0, -2.0, -5.0)
ROOM_HI = (5.0, 2.0, 5.0)


def room_scene(seed: int, n: int, n_keyframes: int = 1, width: int = 1200, height: int = 680,
               f: float = 600.0, n_cap: int | None = None, kf_stride: int = 1):
    """A room-sized map (10 x 4 x 10 m) with keyframes on a smooth random walk.

    With kf_stride k the walk has n_keyframes * k poses and every k-th one is a
    keyframe (keyframes k steps apart).  Returns (params, target_params, cams).
    """
    rng = np.random.default_rng(seed)
    p = draw_gaussians(rng, n, ROOM_LO, ROOM_HI, n_cap)
    tgt = perturb(rng, p, n)
    poses = random_walk(rng, n_keyframes * kf_stride, ROOM_LO, ROOM_HI)[::kf_stride]
    cams = [pinhole(width, height, f, f, width / 2.0, height / 2.0, R, t) for R, t in poses]
    return p, tgt, cams


def mixed_keyframes(seed: int, n_keyframes: int = 32):
    """Keyframes of mixed resolution on one random walk: 640x480 (f=320),
    752x480 (f=376) and 1200x680 (f=600), in the proportions 12:10:10."""
    rng = np.random.default_rng(seed + 7919)
    poses = random_walk(rng, n_keyframes, ROOM_LO, ROOM_HI)
    cams = []
    for i, (R, t) in enumerate(poses):
        j = i * 32 // n_keyframes
        if j < 12:
            w, h, f = 640, 480, 320.0
        elif j < 22:
            w, h, f = 752, 480, 376.0
        else:
            w, h, f = 1200, 680, 600.0
        cams.append(pinhole(w, h, f, f, w / 2.0, h / 2.0, R, t))
    return cams


def smooth_image(rng: np.random.Generator, height: int, width: int, channels: int = 3) -> np.ndarray:
    """A seeded smooth random image in [0, 1] (sum of a few low-frequency cosines)."""
    yy, xx = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    img = np.zeros((channels, height, width), np.float64)
    for c in range(channels):
        acc = np.full((height, width), 0.5)
        for _ in range(6):
            kx, ky = rng.uniform(0.0, 0.08, size=2)
            ph = rng.uniform(0, 2 * np.pi)
            acc += rng.uniform(0.02, 0.12) * np.cos(kx * xx + ky * yy + ph)
        img[c] = np.clip(acc, 0.0, 1.0)
    return img.astype(np.float32)


def densify_case(seed: int, n: int, n_views: int = 2, extent: float = 10.0, n_cap: int | None = None,
                 grad_median: float = 2e-4):
    """Inputs of the densification rule for a map of ``n`` Gaussians.

    The laws straddle the rule's thresholds for a scene of the given extent:
    log-scales ~ N(ln(0.01 extent), 1) per axis (so both clones and splits
    occur, and a few primitives exceed 0.1 extent), opacity logits ~ N(-1, 2.5)
    (a few percent below logit(0.005)), visit counts uniform on 0..8 and mean
    gradient norms log-normal around ``grad_median`` (sigma 0.7).  Also per-view 2D-gradient
    accumulators ``[n_views, n_cap, 9]`` with about a third of the records
    zero and a tenth carrying colour gradients only, the views' level-0 sizes,
    Adam moments and the split noise ``[6, n_cap]``.  Returns a dict.
    """
    rng = np.random.default_rng(seed + 104729)
    n_cap = pad_cap(n) if n_cap is None else n_cap
    p = draw_gaussians(rng, n, ROOM_LO, ROOM_HI, n_cap)
    p[3:6, :n] = rng.normal(math.log(0.01 * extent), 1.0, size=(3, n))
    p[10, :n] = rng.normal(-1.0, 2.5, size=n)
    m = np.zeros((NROWS, n_cap), np.float32)
    v = np.zeros((NROWS, n_cap), np.float32)
    m[:, :n] = rng.normal(0.0, 1e-3, size=(NROWS, n))
    v[:, :n] = rng.uniform(0.0, 1e-6, size=(NROWS, n))
    stats = np.zeros((2, n_cap), np.float32)
    visits = rng.integers(0, 9, size=n).astype(np.float32)
    mean = np.exp(rng.normal(math.log(grad_median), 0.7, size=n))
    stats[0, :n] = (visits * mean).astype(np.float32)
    stats[1, :n] = visits
    noise = np.zeros((6, n_cap), np.float32)
    noise[:, :n] = rng.normal(size=(6, n))
    acc = np.zeros((n_views, n_cap, 9), np.float32)
    vals = rng.normal(0.0, 1e-6, size=(n_views, n, 9))
    kind = rng.uniform(size=(n_views, n))
    vals[kind < 0.33] = 0.0
    colour_only = (kind >= 0.33) & (kind < 0.43)
    vals[..., :6][colour_only] = 0.0
    acc[:, :n] = vals
    sizes = [((1200, 680), (640, 480), (752, 480))[i % 3] for i in range(n_views)]
    return dict(params=p, m=m, v=v, stats=stats, noise=noise, acc=acc, sizes=sizes, n=n, n_cap=n_cap,
                extent=extent)


DEGENERATE_KINDS = {"normal": 200, "behind": 60, "near": 40, "near_plane": 80, "offscreen": 60,
                    "huge": 12, "needle": 100, "faint": 60, "opaque": 40, "dark": 80, "tie": 6}


def degenerate_scene(seed: int = 0):
    """Edge cases of projection and compositing on a ragged 97x61 camera (f=80).

    ``DEGENERATE_KINDS`` gives the number of primitives of each kind, all in
    front of the camera at depth 1.5-3 m unless stated: normal (as
    ``draw_gaussians``); behind (depth -3 to -0.05: culled); near (depth
    0.21-0.5, small: large footprints); near_plane (depth within 0.002-0.03 of
    0.2 on either side: culled or kept); offscreen (image coordinates up to
    three half-widths outside the view, 0.3-1 m wide: the field-of-view clamp
    of the projection Jacobian); huge (1-3 m wide, opacity 0.03-0.08: every
    tile); needle (one axis 1000x the other two); faint (opacity below 1/255:
    never composited); opaque (opacity logit 10-14: the 0.99 clamp and early
    stops); dark (negative colour before the clamp); tie (exact copies of
    normal primitives: equal depths, ordered by index).

    Returns (params, cam, kinds) with ``kinds`` the kind index per column.
    """
    rng = np.random.default_rng(seed)
    W, H, f = 97, 61, 80.0
    cam = pinhole(W, H, f, f, W / 2.0 + 0.3, H / 2.0 - 0.2)
    names = list(DEGENERATE_KINDS)
    counts = [DEGENERATE_KINDS[k] for k in names]
    n = sum(counts)
    p = np.zeros((NROWS, pad_cap(n)), np.float32)
    kinds = np.repeat(np.arange(len(names)), counts)
    starts = np.concatenate([[0], np.cumsum(counts)])

    def in_view(m, z, margin=1.0):
        u = rng.uniform(-margin, margin, m) * (W / 2.0) / f
        v = rng.uniform(-margin, margin, m) * (H / 2.0) / f
        return np.stack([u * z, v * z, z])

    base = draw_gaussians(rng, n, (0, 0, 0), (1, 1, 1))[:, :n]
    mu = np.zeros((3, n))
    for i, name in enumerate(names):
        k = counts[i]
        cols = slice(starts[i], starts[i + 1])
        z = rng.uniform(1.5, 3.0, k)
        if name == "behind":
            z = rng.uniform(-3.0, -0.05, k)
        elif name == "near":
            z = rng.uniform(0.21, 0.5, k)
        elif name == "near_plane":
            z = 0.2 + rng.choice([-1.0, 1.0], k) * rng.uniform(0.002, 0.03, k)
        mu[:, cols] = in_view(k, z, 3.0 if name == "offscreen" else 1.0)
        if name == "behind":
            mu[:2, cols] = rng.uniform(-1, 1, (2, k))
        if name == "near":
            base[3:6, cols] = rng.normal(-5.0, 0.3, (3, k))
        elif name == "offscreen":
            base[3:6, cols] = np.log(rng.uniform(0.3, 1.0, (3, k)))
        elif name == "huge":
            base[3:6, cols] = np.log(rng.uniform(1.0, 3.0, (3, k)))
            base[10, cols] = rng.uniform(-3.5, -2.5, k)
        elif name == "needle":
            base[3, cols] = rng.normal(-2.0, 0.2, k)
            base[4:6, cols] = base[3, cols] - math.log(1000.0)
        elif name == "faint":
            base[10, cols] = rng.uniform(-9.0, -6.0, k)
        elif name == "opaque":
            base[10, cols] = rng.uniform(10.0, 14.0, k)
            base[3:6, cols] = rng.normal(-4.0, 0.3, (3, k))
        elif name == "dark":
            base[11:14, cols] = rng.normal(-2.0, 0.3, (3, k))
    p[:, :n] = base
    p[0:3, :n] = mu
    t = names.index("tie")
    src = rng.choice(counts[0], counts[t], replace=False)   # copies of normal primitives
    p[:, starts[t]:starts[t + 1]] = p[:, src]
    return p, cam, kinds
