"""Loop-closure correction of the primitives: FP64 oracle (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use this module; it shares no code with the GPU library.

Section 3.5: when a loop is closed, the keyframes and map points are moved by
similarity corrections, and the hyper primitives follow.  A similarity
x' = s R x + t moves a primitive's centre to s R mu + t, turns its frame
(quaternion q_R * q), scales it (log-scale + ln s), keeps its opacity, and
turns its view-dependent colour with it: the new colour seen along d equals
the old colour seen along R^T d.  For real spherical harmonics this is a
linear map per band: with D_l(R) defined by Y_l(R^T d) = D_l(R) Y_l(d), the
band-l coefficients c_l become D_l(R)^T c_l.

Here D_l(R) is computed from its definition as an inner product on the
sphere, D_l[i][j] = integral of Y_li(R^T d) Y_lj(d) over the sphere (the
basis is orthonormal), with a product Gauss-Legendre (in cos theta) x
uniform (in phi) rule that integrates these degree <= 6 polynomials exactly.
The basis values come from the oracle's own real-SH basis.
"""

from __future__ import annotations

import math

import numpy as np

from . import sh_basis

BANDS = [(1, 1, 4), (2, 4, 9), (3, 9, 16)]   # (l, first k, end k)


def quat_rotation(q) -> np.ndarray:
    """Rotation matrix of the normalised quaternion (w, x, y, z)."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def quat_mul(a, b) -> np.ndarray:
    """Hamilton product a * b of quaternions (w, x, y, z)."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def _sphere_rule(n_theta: int = 8, n_phi: int = 16):
    """Nodes (unit vectors) and weights of the product rule on the sphere."""
    ct, wt = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * math.pi * np.arange(n_phi) / n_phi
    dirs, wts = [], []
    for c, w in zip(ct, wt):
        s = math.sqrt(max(0.0, 1 - c * c))
        for p in phi:
            dirs.append((s * math.cos(p), s * math.sin(p), c))
            wts.append(w * 2 * math.pi / n_phi)
    return np.array(dirs), np.array(wts)


def sh_rotation(R) -> list:
    """[D_1, D_2, D_3]: Y_l(R^T d) = D_l(R) Y_l(d) for the real SH bands 1..3."""
    R = np.asarray(R, np.float64)
    dirs, wts = _sphere_rule()
    Yd = np.array([sh_basis(d)[0] for d in dirs])            # [nodes, 16]
    Yr = np.array([sh_basis(R.T @ d)[0] for d in dirs])       # values at R^T d
    out = []
    for _, a, b in BANDS:
        out.append((Yr[:, a:b] * wts[:, None]).T @ Yd[:, a:b])
    return out


def moved_camera(cam: dict, sim) -> dict:
    """The camera that sees the transformed world as `cam` saw the old one:
    world-to-camera R_c R^T, s t_c - R_c R^T t (intrinsics unchanged)."""
    q, t, s = sim
    R = quat_rotation(q)
    Rc = np.asarray(cam["R"], np.float64)
    tc = np.asarray(cam["t"], np.float64)
    out = dict(cam)
    out["R"] = Rc @ R.T
    out["t"] = s * tc - Rc @ R.T @ np.asarray(t, np.float64)
    return out


def apply_sim3(P, n: int, sims, assign=None) -> np.ndarray:
    """Primitives 0..n-1 of P ([59, >=n]) moved by sims[assign[g]] (each
    ((w, x, y, z), t, s)); assign None means transform 0 for all; an index
    outside [0, len(sims)) leaves the primitive unchanged.  FP64 result."""
    P = np.array(P, np.float64)
    mats = [(quat_rotation(q), np.asarray(q, np.float64) / np.linalg.norm(q), np.asarray(t, np.float64),
             float(s), sh_rotation(quat_rotation(q))) for (q, t, s) in sims]
    for g in range(n):
        k = 0 if assign is None else int(assign[g])
        if k < 0 or k >= len(sims):
            continue
        R, qn, t, s, D = mats[k]
        P[0:3, g] = s * (R @ P[0:3, g]) + t
        P[3:6, g] = P[3:6, g] + math.log(s)
        P[6:10, g] = quat_mul(qn, P[6:10, g])
        for ch in range(3):
            for (l, a, b), Dl in zip(BANDS, D):
                rows = [11 + 3 * k2 + ch for k2 in range(a, b)]
                P[rows, g] = Dl.T @ P[rows, g]
    return P
