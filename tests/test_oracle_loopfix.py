"""Pins of the loop-closure oracle (Section 3.5: primitives follow the
similarity corrections of a closed loop): the SH band rotations against a
closed form, the group law and their definition; the whole transform
against rendering (a moved map seen from the correspondingly moved camera
renders the same image)."""

import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenes
from oracle import loopfix as lf


def _rot(seed):
    return Rotation.random(random_state=seed).as_matrix()


def test_band1_closed_form():
    """Band 1 is (-y, z, -x) up to a constant, so D_1 = S R^T S^T."""
    S = np.array([[0, -1, 0], [0, 0, 1], [-1, 0, 0]], float)
    for seed in range(3):
        R = _rot(seed)
        np.testing.assert_allclose(lf.sh_rotation(R)[0], S @ R.T @ S.T, atol=1e-13)


def test_group_law_orthogonality_identity():
    R1, R2 = _rot(10), _rot(11)
    D1, D2, D12 = lf.sh_rotation(R1), lf.sh_rotation(R2), lf.sh_rotation(R1 @ R2)
    for a, b, ab in zip(D1, D2, D12):
        np.testing.assert_allclose(ab, b @ a, atol=1e-12)          # D(R1 R2) = D(R2) D(R1)
        np.testing.assert_allclose(a @ a.T, np.eye(len(a)), atol=1e-12)
    for Dl in lf.sh_rotation(np.eye(3)):
        np.testing.assert_allclose(Dl, np.eye(len(Dl)), atol=1e-13)


def test_definition_at_random_directions():
    import oracle

    R = _rot(3)
    D = lf.sh_rotation(R)
    rng = np.random.default_rng(0)
    for _ in range(50):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        Yd = oracle.sh_basis(d)[0]
        Yr = oracle.sh_basis(R.T @ d)[0]
        for (_, a, b), Dl in zip(lf.BANDS, D):
            np.testing.assert_allclose(Yr[a:b], Dl @ Yd[a:b], atol=1e-13)


def test_quaternion_product_composes_rotations():
    a, b = Rotation.random(random_state=4), Rotation.random(random_state=5)
    qa = a.as_quat()[[3, 0, 1, 2]]
    qb = b.as_quat()[[3, 0, 1, 2]]
    np.testing.assert_allclose(lf.quat_rotation(lf.quat_mul(qa, qb)), (a * b).as_matrix(), atol=1e-13)
    np.testing.assert_allclose(lf.quat_rotation(qa), a.as_matrix(), atol=1e-13)


@pytest.mark.parametrize("scale", [1.0, 1.7, 0.8])
def test_moved_map_renders_like_the_moved_camera(orc, scale):
    """Render(apply(P), moved camera) == Render(P, camera): pins the centre,
    frame, scale and colour (SH) transforms together; the scene keeps every
    depth far from the near plane at either scale."""
    p, _, cam = scenes.tiny_scene(1, n=1500)
    q = Rotation.from_rotvec([0.3, -0.5, 0.9]).as_quat()[[3, 0, 1, 2]]
    sim = (q, np.array([0.4, -1.2, 2.5]), scale)
    moved = lf.apply_sim3(p, 1500, [sim])
    cam2 = lf.moved_camera(cam, sim)
    a = orc.render(p, 1500, cam)
    b = orc.render(moved, 1500, cam2)
    assert np.abs(a["img"] - b["img"]).max() < 1e-9
    assert np.abs(a["T"] - b["T"]).max() < 1e-9
    assert np.array_equal(a["n_contrib"], b["n_contrib"])
    # the view-dependent colour matters here: without the SH rotation the
    # images differ
    wrong = moved.copy()
    wrong[14:59, :1500] = p[14:59, :1500]
    c = orc.render(wrong, 1500, cam2)
    assert np.abs(a["img"] - c["img"]).max() > 1e-3


def test_assignment_and_identity():
    c = scenes.densify_case(0, 300)
    P = c["params"][:, :300]
    ident = ((1.0, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 1.0)
    np.testing.assert_allclose(lf.apply_sim3(P, 300, [ident]), P, atol=1e-15)
    q = Rotation.random(random_state=2).as_quat()[[3, 0, 1, 2]]
    sims = [ident, (q, (1.0, 2.0, 3.0), 2.0)]
    assign = np.array([1, -1, 0, 2, 1] * 60, np.int32)
    out = lf.apply_sim3(P, 300, sims, assign)
    unchanged = (assign < 0) | (assign >= 2) | (assign == 0)
    np.testing.assert_allclose(out[:, unchanged], P[:, unchanged], atol=1e-15)
    moved = assign == 1
    R = lf.quat_rotation(q)
    np.testing.assert_allclose(out[0:3, moved], 2.0 * R @ P[0:3, moved] + np.array([[1.0], [2.0], [3.0]]),
                               atol=1e-12)
    np.testing.assert_allclose(out[3:6, moved], P[3:6, moved] + math.log(2.0), atol=1e-12)
    np.testing.assert_allclose(out[10], P[10], atol=0)
    np.testing.assert_allclose(out[11:14], P[11:14], atol=1e-15)   # band 0 does not turn
