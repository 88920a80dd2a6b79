"""Pins of the oracle's projection step (the 3D Gaussian splat G of Eq. 3, Section 3.3).

Each check compares the oracle against something other than itself: a closed
form computed independently here with numpy and scipy's rotation routine, an
on-axis special case, culling rules, and scale invariance of the image.
"""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenes

DIL = 0.3


def _random_camera(rng, W=160, H=120):
    R = Rotation.from_rotvec(rng.normal(size=3) * 0.3).as_matrix()
    t = rng.normal(size=3) * 0.2
    return scenes.pinhole(W, H, 140.0, 150.0, 81.0, 57.0, R, t)


def _scene_in_front(rng, cam, n):
    """Gaussians placed 2-5 m in front of the camera."""
    p = np.zeros((59, scenes.pad_cap(n)), np.float64)
    xc = np.stack([rng.uniform(-1, 1, n), rng.uniform(-0.8, 0.8, n), rng.uniform(2, 5, n)], 1)
    R = np.asarray(cam["R"], np.float64)
    t = np.asarray(cam["t"], np.float64)
    mu = (xc - t) @ R   # R^T (xc - t)
    p[0:3, :n] = mu.T
    p[3:6, :n] = rng.normal(-2.5, 0.5, (3, n))
    p[6:10, :n] = rng.normal(size=(4, n))          # unnormalised on purpose
    p[10, :n] = rng.normal(size=n)
    p[11:59, :n] = rng.normal(0, 0.2, (48, n))
    return p


def _closed_form(p, g, cam):
    """Sigma2D = J W Sigma W^T J^T, with scipy's quaternion-to-matrix (scalar last)."""
    mu = p[0:3, g]
    s = np.exp(p[3:6, g])
    q = p[6:10, g]
    Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    Sig = Rq @ np.diag(s ** 2) @ Rq.T
    W = np.asarray(cam["R"], np.float64)
    xc = W @ mu + np.asarray(cam["t"], np.float64)
    x, y, z = xc
    fx, fy = cam["fx"], cam["fy"]
    limx = 1.3 * cam["width"] / (2 * fx)
    limy = 1.3 * cam["height"] / (2 * fy)
    u = np.clip(x / z, -limx, limx)
    v = np.clip(y / z, -limy, limy)
    J = np.array([[fx / z, 0, -fx * u / z], [0, fy / z, -fy * v / z]])
    S2 = J @ W @ Sig @ W.T @ J.T
    m = np.array([fx * x / z + cam["cx"], fy * y / z + cam["cy"]])
    return S2, m, z


def test_cov2d_matches_closed_form(orc):
    rng = np.random.default_rng(11)
    cam = _random_camera(rng)
    n = 200
    p = _scene_in_front(rng, cam, n)
    rec = orc.preprocess(p, n, cam)
    assert rec[:, 0].all()
    for g in range(n):
        S2, m, z = _closed_form(p, g, cam)
        got = np.array([[rec[g, 14] - DIL, rec[g, 15]], [rec[g, 15], rec[g, 16] - DIL]])
        np.testing.assert_allclose(got, S2, rtol=1e-10, atol=1e-10 * np.abs(S2).max())
        np.testing.assert_allclose(rec[g, 1:3], m, rtol=1e-12)
        assert rec[g, 3] == pytest.approx(z, rel=1e-13)
        # conic is the inverse of the dilated covariance
        K = np.array([[rec[g, 4], rec[g, 5]], [rec[g, 5], rec[g, 6]]])
        np.testing.assert_allclose(K @ (S2 + DIL * np.eye(2)), np.eye(2), atol=1e-10)


def test_fov_clamp_freezes_jacobian_off_axis(orc):
    """A Gaussian far outside the frustum uses the clamped direction in J."""
    cam = scenes.pinhole(100, 80, 100.0)
    p = np.zeros((59, 256))
    p[0:3, 0] = [3.0, -2.5, 2.0]      # u = 1.5 > 1.3*0.5, v = -1.25 < -1.3*0.4
    p[3:6, 0] = [-1.0, -1.5, -2.0]
    p[6:10, 0] = [0.9, 0.1, -0.3, 0.2]
    rec = orc.preprocess(p, 1, cam)
    S2, _, _ = _closed_form(p, 0, cam)
    np.testing.assert_allclose([rec[0, 14] - DIL, rec[0, 15], rec[0, 16] - DIL],
                               [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-11)


def test_isotropic_on_axis():
    """Isotropic Gaussian on the optical axis: Sigma2D = (f s / z)^2 I + 0.3 I, centre (cx, cy)."""
    import oracle

    cam = scenes.pinhole(128, 128, 128.0, 128.0, 64.0, 64.0)
    p = np.zeros((59, 256))
    z, s = 3.0, 0.05
    p[0:3, 0] = [0, 0, z]
    p[3:6, 0] = np.log(s)
    p[6:10, 0] = [0.3, -0.5, 0.7, 0.1]   # any rotation: isotropic
    rec = oracle.preprocess(p, 1, cam)
    expect = (128.0 * s / z) ** 2 + DIL
    assert rec[0, 14] == pytest.approx(expect, rel=1e-12)
    assert rec[0, 16] == pytest.approx(expect, rel=1e-12)
    assert abs(rec[0, 15]) < 1e-14
    assert rec[0, 1] == 64.0 and rec[0, 2] == 64.0


def test_near_plane_cull(orc):
    cam = scenes.pinhole(64, 64, 64.0)
    p = np.zeros((59, 256))
    p[6, :3] = 1.0
    p[0:3, 0] = [0, 0, 0.2]      # exactly on z_near: culled
    p[0:3, 1] = [0, 0, 0.2001]   # just beyond: kept
    p[0:3, 2] = [0, 0, -1.0]     # behind
    rec = orc.preprocess(p, 3, cam)
    assert list(rec[:, 0]) == [0.0, 1.0, 0.0]


def test_scale_invariance_of_image(orc):
    """Scaling means, scales and camera translation by k leaves the image unchanged."""
    p, _, cam = scenes.tiny_scene(3, n=300)
    p = p.astype(np.float64)
    cam = dict(cam)
    cam["t"] = np.array([0.1, -0.05, 0.2])
    k = 2.5
    p2 = p.copy()
    p2[0:3] *= k
    p2[3:6, :300] += np.log(k)
    cam2 = dict(cam)
    cam2["t"] = cam["t"] * k
    a = orc.render(p, 300, cam)
    b = orc.render(p2, 300, cam2)
    np.testing.assert_allclose(a["img"], b["img"], atol=1e-10)
    assert np.array_equal(a["n_contrib"], b["n_contrib"])


def test_quaternion_normalisation(orc):
    """Scaling the raw quaternion leaves every record unchanged."""
    rng = np.random.default_rng(5)
    cam = _random_camera(rng)
    p = _scene_in_front(rng, cam, 50)
    p2 = p.copy()
    p2[6:10] *= 3.7
    np.testing.assert_allclose(orc.preprocess(p, 50, cam), orc.preprocess(p2, 50, cam), rtol=1e-12,
                               atol=1e-14)


def test_degenerate_scene_rules(orc):
    """Each kind of the degenerate scene meets the rule it was built to reach
    (camera at the origin looking along +z, so a primitive's depth is its z):
    culled exactly when z <= 0.2; faint primitives (opacity below 1/255) in no
    pixel's list; field-of-view clamp for off-screen ones (|x/z| beyond 1.3
    half-widths); colour clamped for dark ones; an exact copy right behind its
    source in every pixel list that holds both."""
    p, cam, kinds = scenes.degenerate_scene(0)
    n = kinds.size
    names = list(scenes.DEGENERATE_KINDS)
    k = {nm: np.nonzero(kinds == i)[0] for i, nm in enumerate(names)}
    rec = orc.preprocess(p, n, cam)
    z = p[2, :n].astype(np.float64)
    assert np.array_equal(rec[:, 0] > 0, z > 0.2)
    assert np.any(z[k["near_plane"]] > 0.2) and np.any(z[k["near_plane"]] <= 0.2)
    assert not np.any(rec[k["behind"], 0])
    u = np.abs(p[0, :n] / p[2, :n]).astype(np.float64)
    limx = 1.3 * 0.5 * cam["width"] / cam["fx"]
    assert np.sum(u[k["offscreen"]] > limx) >= 10
    assert np.all(rec[k["dark"]][:, 11:14].sum(axis=1) >= 1)   # some channel clamped
    faint = set(k["faint"].tolist())
    pairs_seen = 0
    src_of = {}
    t = k["tie"]
    for c in t:
        same = np.nonzero(np.all(p[:, :n] == p[:, [c]], axis=0))[0]
        src_of[int(c)] = int(same[0])
    for py in range(0, cam["height"], 4):
        for px in range(0, cam["width"], 4):
            ids = orc.pixel_list(p, n, cam, px, py).tolist()
            assert not faint.intersection(ids)
            for c, s in src_of.items():
                if c in ids and s in ids:
                    assert ids.index(c) == ids.index(s) + 1
                    pairs_seen += 1
    assert pairs_seen > 0
