"""Gradient-driven densification of the map: FP64 oracle (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use this module; it shares no code with the GPU library.

Section 3.3.1: besides the geometry-based densification, the photorealistic
mapper splits or clones primitives whose loss gradients are large, following
the adaptive density control of 3D Gaussian splatting (Kerbl et al. 2023,
Sec. 5.2).  That rule, restated:

* statistic: per primitive, the running mean over (iteration, view) visits of
  the norm of the loss gradient with respect to its projected 2D mean, taken
  in normalised device coordinates (x_ndc = (2 x_pix + 1) / W - 1, so
  dL/dx_ndc = dL/dx_pix * W / 2);
* a primitive whose mean reaches ``grad_threshold`` is densified: if its
  largest scale is at most ``percent_dense * extent`` it is cloned (an
  identical copy is added), otherwise it is split into two children whose
  centres are drawn from the primitive's own 3D Gaussian and whose scales are
  the parent's divided by 1.6; the parent is removed;
* primitives (originals and newly made ones alike) whose opacity is below
  ``min_opacity`` or whose largest scale exceeds ``big_fraction * extent`` are
  removed;
* new primitives start with zero optimiser moments; survivors keep theirs.

Readings fixed here (the design notes list them): a view counts as a visit
when the primitive's record received any nonzero 2D gradient in it; the
scale tests compare log-scales with the logarithm of the threshold and the
opacity test compares the logit with the logit of ``min_opacity``, all in
float32 (a floating-point comparison that decides a discrete outcome is made
in the kernel's precision); the output keeps the surviving originals in
order, followed, for each original in order, by its clone or its two
children (child 0 from noise rows 0-2, child 1 from rows 3-5).
"""

from __future__ import annotations

import math

import numpy as np

NROWS = 59
F32 = np.float32

# action per original
KEEP, CLONE, SPLIT = 0, 1, 2


def densify_rule(extent: float, grad_threshold: float = 2e-4, percent_dense: float = 0.01,
                 min_opacity: float = 0.005, big_fraction: float | None = 0.1,
                 shrink: float = 1.6) -> dict:
    """The float32 thresholds of the rule for a scene of the given extent."""
    return dict(
        grad_threshold=F32(grad_threshold),
        log_dense=F32(math.log(percent_dense * extent)),
        log_big=F32(math.inf if big_fraction is None else math.log(big_fraction * extent)),
        logit_min=F32(math.log(min_opacity / (1.0 - min_opacity))),
        log_shrink=F32(math.log(shrink)),
        shrink=float(shrink),
    )


def densify_stats(acc, sizes, stats=None) -> np.ndarray:
    """Adds one iteration's visits to the statistic.

    acc: per-view 2D gradients ``[n_views, n, 9]`` (d mean x, d mean y in
    level-0 pixels, then the other seven values of a record); sizes: the
    level-0 ``(width, height)`` of each view.  Returns ``[2, n]`` float64:
    row 0 the summed gradient norms in NDC units, row 1 the visit counts.
    """
    acc = np.asarray(acc, np.float64)
    nv, n = acc.shape[0], acc.shape[1]
    out = np.zeros((2, n), np.float64) if stats is None else np.array(stats, np.float64)
    for v in range(nv):
        W, H = sizes[v]
        visited = np.any(acc[v] != 0.0, axis=1)
        gx = acc[v, :, 0] * (0.5 * W)
        gy = acc[v, :, 1] * (0.5 * H)
        out[0] += np.where(visited, np.sqrt(gx * gx + gy * gy), 0.0)
        out[1] += visited
    return out


def quat_rotation(q) -> np.ndarray:
    """Rotation matrix of the normalised quaternion (w, x, y, z)."""
    q = np.asarray(q, np.float64)
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def decide(P, stats, n: int, rule: dict):
    """Per original: its action (KEEP / CLONE / SPLIT), whether the original
    survives, and how many new primitives it contributes.  Elementwise
    float32 arithmetic and comparisons (IEEE, as on the device)."""
    P32 = np.asarray(P, F32)[:, :n]
    s = np.asarray(stats, F32)[:, :n]
    visits = s[1]
    avg = np.zeros(n, F32)
    seen = visits > F32(0)
    avg[seen] = s[0][seen] / visits[seen]
    maxls = np.maximum(np.maximum(P32[3], P32[4]), P32[5])
    faint = P32[10] < rule["logit_min"]
    prune = faint | (maxls > rule["log_big"])
    hot = avg >= rule["grad_threshold"]
    clone = hot & (maxls <= rule["log_dense"])
    split = hot & ~clone
    child_big = (maxls - rule["log_shrink"]).astype(F32) > rule["log_big"]
    action = np.where(clone, CLONE, np.where(split, SPLIT, KEEP)).astype(np.int32)
    keep = ~split & ~prune
    new = np.where(clone & ~prune, 1, 0) + np.where(split & ~(faint | child_big), 2, 0)
    return action, keep, new.astype(np.int32)


# kind of an output column
SURVIVOR, COPY, CHILD0, CHILD1 = 0, 1, 2, 3


def layout(action, keep, new):
    """Source original and kind of every output column: the surviving
    originals in order, then each original's copy or two children."""
    n = len(new)
    kept = np.nonzero(keep)[0]
    src_new = np.repeat(np.arange(n), new)
    first = np.ones(len(src_new), bool)
    first[1:] = src_new[1:] != src_new[:-1]
    kind_new = np.where(action[src_new] == CLONE, COPY, np.where(first, CHILD0, CHILD1))
    src = np.concatenate([kept, src_new]).astype(np.int64)
    kind = np.concatenate([np.full(len(kept), SURVIVOR), kind_new]).astype(np.int32)
    return src, kind


def column(P, m, v, noise, g: int, kind: int, rule: dict):
    """One output column (parameters, m, v) in FP64."""
    p = np.asarray(P[:, g], np.float64).copy()
    if kind == SURVIVOR:
        return p, np.asarray(m[:, g], np.float64), np.asarray(v[:, g], np.float64)
    if kind in (CHILD0, CHILD1):
        c = kind - CHILD0
        R = quat_rotation(p[6:10])
        z = np.asarray(noise[3 * c:3 * c + 3, g], np.float64)
        p[0:3] = p[0:3] + R @ (np.exp(p[3:6]) * z)
        p[3:6] = p[3:6] - math.log(rule["shrink"])
    return p, np.zeros(NROWS), np.zeros(NROWS)


def densify(P, m, v, stats, n: int, noise, rule: dict):
    """Applies the rule.  P, m, v: ``[59, >=n]``; stats ``[2, >=n]``; noise
    ``[6, >=n]`` standard normals (child 0 rows 0-2, child 1 rows 3-5).
    Returns (P_out, m_out, v_out) ``[59, n_out]`` float64 and the counts
    (n_out, cloned, split, pruned originals)."""
    action, keep, new = decide(P, stats, n, rule)
    src, kind = layout(action, keep, new)
    P_out = np.zeros((NROWS, len(src)))
    m_out = np.zeros((NROWS, len(src)))
    v_out = np.zeros((NROWS, len(src)))
    for j in range(len(src)):
        P_out[:, j], m_out[:, j], v_out[:, j] = column(P, m, v, noise, int(src[j]), int(kind[j]), rule)
    counts = dict(n_out=len(src), cloned=int(np.sum((action == CLONE) & (new > 0))),
                  split=int(np.sum(action == SPLIT)),
                  pruned=int(np.sum((action != SPLIT) & ~keep)))
    return P_out, m_out, v_out, counts


def reset_opacity(P, m, v, n: int, max_opacity: float = 0.01):
    """Opacity reset of the same rule: every opacity above ``max_opacity`` is
    lowered to it (logit min(logit, logit(max_opacity)), compared in float32)
    and the opacity row's optimiser moments are cleared."""
    cap = F32(math.log(max_opacity / (1.0 - max_opacity)))
    P = np.array(P, np.float64)
    m = np.array(m, np.float64)
    v = np.array(v, np.float64)
    lo = np.asarray(P[10, :n], F32)
    P[10, :n] = np.where(lo > cap, np.float64(cap), P[10, :n])
    m[10, :n] = 0.0
    v[10, :n] = 0.0
    return P, m, v
