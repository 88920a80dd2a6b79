"""Pins of the oracle's front-to-back compositing (Eq. 3, Section 3.3).

Closed forms (single Gaussian at its centre, an occluding stack with the early
stop), the integral of the splat over the image, monotone transmittance, the
empty scene, the candidate pre-filter against brute force, an independent
pure-numpy per-pixel depth sort on tiny scenes, and invariance under
permutation of the Gaussians and under a rigid motion of scene and camera.
"""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenes

C0 = 1.0 / (2.0 * np.sqrt(np.pi))   # value of the degree-0 real SH


def _blank(n):
    p = np.zeros((59, scenes.pad_cap(n)))
    p[6, :n] = 1.0
    return p


def _logit(o):
    return np.log(o / (1 - o))


def _dc_for(rgb):
    return (np.asarray(rgb, np.float64) - 0.5) / C0


@pytest.mark.parametrize("o", [0.3, 0.7, 0.995])
def test_single_gaussian_centre(orc, o):
    cam = scenes.pinhole(64, 64, 64.0, 64.0, 32.0, 32.0, bg=(0.2, 0.1, 0.4))
    p = _blank(1)
    p[0:3, 0] = [0, 0, 3]
    p[3:6, 0] = np.log(0.05)
    p[10, 0] = _logit(o)
    rgb = np.array([0.9, 0.3, 0.6])
    p[11:14, 0] = _dc_for(rgb)
    r = orc.render(p, 1, cam)
    a = min(0.99, o)
    expect = a * rgb + (1 - a) * np.asarray(cam["bg"], np.float64)
    np.testing.assert_allclose(r["img"][:, 32, 32], expect, rtol=1e-12)
    assert r["n_contrib"][32, 32] == 1
    assert r["T"][32, 32] == pytest.approx(1 - a, rel=1e-12)


def test_occlusion_stack_and_early_stop(orc):
    """alpha 0.99, 0.98, 0.99 on one ray: C = 0.99 c1 + 0.0098 c2 + 2e-4 bg; the third and
    every later Gaussian add nothing because T would fall below 1e-4."""
    cam = scenes.pinhole(33, 33, 33.0, 33.0, 16.0, 16.0, bg=(0.5, 0.25, 1.0))
    n = 5
    p = _blank(n)
    zs = [2.0, 3.0, 4.0, 5.0, 6.0]
    ops = [0.995, 0.98, 0.995, 0.9, 0.5]
    cols = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [0, 1, 1]]
    # store them in scrambled order: depth order must be recovered
    order = [3, 0, 4, 2, 1]
    for col, k in enumerate(order):
        p[0:3, col] = [0, 0, zs[k]]
        p[3:6, col] = np.log(0.1)
        p[10, col] = _logit(ops[k])
        p[11:14, col] = _dc_for(cols[k])
    r = orc.render(p, n, cam)
    c1, c2 = np.array(cols[0], float), np.array(cols[1], float)
    bg = np.asarray(cam["bg"], np.float64)
    expect = 0.99 * c1 + 0.01 * 0.98 * c2 + 0.01 * 0.02 * bg
    np.testing.assert_allclose(r["img"][:, 16, 16], expect, rtol=1e-12)
    assert r["n_contrib"][16, 16] == 2
    assert r["T"][16, 16] == pytest.approx(2e-4, rel=1e-12)
    ids = orc.pixel_list(p, n, cam, 16, 16)
    assert list(ids) == [order.index(0), order.index(1)]


def test_splat_mass_identity(orc):
    """One wide Gaussian (white, bg black): sum over pixels of alpha equals
    2 pi sqrt(det Sigma2D) (o - 1/255), since alpha is counted only where it
    reaches 1/255.  Riemann error of a 15-px-wide splat is far below 1%."""
    cam = scenes.pinhole(256, 256, 256.0, 256.0, 128.3, 127.6)
    p = _blank(1)
    p[0:3, 0] = [0.01, -0.02, 2.0]
    p[3:6, 0] = np.log([0.12, 0.08, 0.1])
    p[6:10, 0] = [0.9, 0.2, 0.3, -0.1]
    o = 0.6
    p[10, 0] = _logit(o)
    p[11:14, 0] = _dc_for([1, 1, 1])
    rec = orc.preprocess(p, 1, cam)
    det = rec[0, 14] * rec[0, 16] - rec[0, 15] ** 2
    r = orc.render(p, 1, cam)
    mass = r["img"][0].sum()
    assert mass == pytest.approx(2 * np.pi * np.sqrt(det) * (o - 1 / 255), rel=2e-3)
    # without the cutoff the same sum would be 2 pi sqrt(det) o: the -1/255 term is resolved
    assert abs(mass - 2 * np.pi * np.sqrt(det) * o) > 50 * abs(mass - 2 * np.pi * np.sqrt(det) * (o - 1 / 255))


def test_transmittance_bounds_and_empty(orc):
    p, _, cam = scenes.tiny_scene(0)
    r = orc.render(p, 2000, cam)
    assert r["T"].min() >= 1e-4 and r["T"].max() <= 1.0
    assert np.all(r["T"][r["n_contrib"] == 0] == 1.0)
    assert r["counts"]["composited"] == r["n_contrib"].sum()
    # zero opacity everywhere: background and T = 1
    q = p.copy()
    q[10] = -50.0
    cam2 = dict(cam, bg=np.array([0.1, 0.2, 0.3]))
    e = orc.render(q, 2000, cam2)
    assert np.all(e["T"] == 1.0) and np.all(e["n_contrib"] == 0)
    bg = np.asarray(cam2["bg"], np.float64)
    np.testing.assert_array_equal(e["img"], np.broadcast_to(bg[:, None, None], e["img"].shape))
    z = orc.render(p, 0, cam2)
    assert np.all(z["T"] == 1.0)


def test_transmittance_is_product_along_list(orc):
    """T_final equals the product of (1 - alpha) over the pixel's list, and the list is
    sorted by depth."""
    p, _, cam = scenes.tiny_scene(1, n=400)
    r = orc.render(p, 400, cam)
    rec = orc.preprocess(p, 400, cam)
    rng = np.random.default_rng(0)
    for _ in range(25):
        x, y = rng.integers(0, 128, 2)
        ids = orc.pixel_list(p, 400, cam, x, y)
        dx = rec[ids, 1] - x
        dy = rec[ids, 2] - y
        pw = -0.5 * (rec[ids, 4] * dx * dx + rec[ids, 6] * dy * dy) - rec[ids, 5] * dx * dy
        a = np.minimum(0.99, rec[ids, 7] * np.exp(pw))
        assert np.all(np.diff(rec[ids, 3]) >= 0)
        assert r["T"][y, x] == pytest.approx(np.prod(1 - a), rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_prefilter_equals_brute_force(orc, seed):
    p, _, cam = scenes.tiny_scene(seed, n=600)
    a = orc.render(p, 600, cam, prune=True)
    b = orc.render(p, 600, cam, prune=False)
    assert np.array_equal(a["img"], b["img"])
    assert np.array_equal(a["T"], b["T"])
    assert np.array_equal(a["n_contrib"], b["n_contrib"])


def _numpy_brute_force(rec, cam, n):
    """Independent per-pixel depth sort + composite from the projection records."""
    H, W = cam["height"], cam["width"]
    img = np.zeros((3, H, W))
    T_out = np.ones((H, W))
    bg = np.asarray(cam["bg"], np.float64)
    for y in range(H):
        for x in range(W):
            items = []
            for g in range(n):
                if rec[g, 0] == 0:
                    continue
                dx, dy = rec[g, 1] - x, rec[g, 2] - y
                pw = -0.5 * (rec[g, 4] * dx * dx + rec[g, 6] * dy * dy) - rec[g, 5] * dx * dy
                at = rec[g, 7] * np.exp(pw)
                if at >= 1 / 255:
                    items.append((rec[g, 3], g, min(0.99, at)))
            items.sort()
            T, C = 1.0, np.zeros(3)
            for _, g, a in items:
                Tn = T * (1 - a)
                if Tn < 1e-4:
                    break
                C += a * T * rec[g, 8:11]
                T = Tn
            img[:, y, x] = C + T * bg
            T_out[y, x] = T
    return img, T_out


@pytest.mark.parametrize("seed", [0, 1])
def test_numpy_brute_force_tiny(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n = 48
    p = _blank(n)
    p[0:3, :n] = np.stack([rng.uniform(-0.4, 0.4, n), rng.uniform(-0.4, 0.4, n), rng.uniform(1.5, 2.5, n)])
    p[3:6, :n] = rng.normal(-2.6, 0.4, (3, n))
    p[6:10, :n] = rng.normal(size=(4, n))
    p[10, :n] = rng.normal(1.0, 1.5, n)
    p[11:59, :n] = rng.normal(0, 0.3, (48, n))
    cam = scenes.pinhole(32, 32, 40.0, 40.0, 16.0, 15.0, bg=(0.3, 0.6, 0.1))
    r = orc.render(p, n, cam, prune=False)
    rec = orc.preprocess(p, n, cam)
    img, T = _numpy_brute_force(rec, cam, n)
    np.testing.assert_allclose(r["img"], img, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(r["T"], T, rtol=1e-13)
    assert r["n_contrib"].max() > 3   # the scene has real overlap


def test_permutation_invariance(orc):
    p, _, cam = scenes.tiny_scene(4, n=500)
    perm = np.random.default_rng(9).permutation(500)
    q = p.copy()
    q[:, :500] = p[:, perm]
    a = orc.render(p, 500, cam)
    b = orc.render(q, 500, cam)
    assert np.array_equal(a["img"], b["img"]) and np.array_equal(a["n_contrib"], b["n_contrib"])


def test_rigid_motion_invariance_dc_only(orc):
    """Moving scene and camera by the same rigid motion changes nothing (DC-only SH)."""
    p, _, cam = scenes.tiny_scene(5, n=400)
    p = p.astype(np.float64)
    p[14:59] = 0.0
    rg = Rotation.from_rotvec([0.3, -0.7, 0.2])
    tg = np.array([1.5, -0.4, 2.0])
    q = p.copy()
    q[0:3, :400] = (rg.as_matrix() @ p[0:3, :400]) + tg[:, None]
    quats = p[6:10, :400].T                       # (w, x, y, z)
    rot = rg * Rotation.from_quat(quats[:, [1, 2, 3, 0]])
    xyzw = rot.as_quat()
    q[6:10, :400] = xyzw[:, [3, 0, 1, 2]].T
    cam2 = dict(cam)
    R = np.asarray(cam["R"], np.float64) @ rg.as_matrix().T
    cam2["R"] = R
    cam2["t"] = np.asarray(cam["t"], np.float64) - R @ tg
    a = orc.render(p, 400, cam)
    b = orc.render(q, 400, cam2)
    np.testing.assert_allclose(a["img"], b["img"], atol=1e-9)
