"""Tile shapes (tile_w x 256/tile_w pixels, picked by the autotuner): every
shape renders within the parity bar of the oracle on every target and
level, and gradients match the oracle for every shape.  A pixel composites
the same Gaussians in the same order whatever tile holds it, but the staged
offsets are relative to the tile's origin, so their FP32 rounding (and a
near-cutoff decision now and then) depends on the shape: shapes agree to
FP32 rounding, not bitwise (batch and wave choices for one shape are bitwise
equal, see the launch-shape test)."""

import numpy as np
import pytest
import torch

import scenes
from tests.gpu_util import check_gradients, plan_for, require_gpu

pytestmark = pytest.mark.gpu

WIDTHS = (8, 16, 32)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


RAGGED = scenes.pinhole(150, 110, 130.0, 125.0, 71.3, 52.6, R=np.eye(3), t=[0.05, -0.03, 0.1],
                        bg=(0.2, 0.4, 0.1))


def _scene():
    p, tp, _ = scenes.tiny_scene(3, n=1500)
    cam2 = scenes.pinhole(97, 61, 90.0, 90.0, 45.0, 30.0, R=np.eye(3), t=[-0.02, 0.04, 0.0])
    return p, tp, 1500, [RAGGED, cam2]


@pytest.mark.parametrize("tw", WIDTHS)
def test_forward_matches_oracle_for_tile_shape(orc, tw):
    from tests.gpu_util import compare_image

    p, _, n, cams = _scene()
    plan = plan_for(cams, levels=(0, 1, 2), n_cap=p.shape[1], tile_w=tw)
    plan.render(_dev(p), n, with_ncontrib=True)
    torch.cuda.synchronize()
    assert not plan.overflowed()
    for i, (v, l, _, _) in enumerate(plan.specs):
        cam = scenes.level_camera(cams[v], l)
        o = orc.render(p, n, cam)
        img = plan.image(plan.rgb, i).cpu().numpy()
        T = plan.plane(plan.T, i).cpu().numpy()
        m_img, m_T, n_amb, _, ok = compare_image(img, T, o)
        print(f"tile_w {tw} target {i}: {plan.total_tiles} tiles, max|dI|={m_img:.2e} ambiguous={n_amb}")
        assert m_img <= 1e-4 and m_T <= 1e-4
        strict = o["amb"] == 0
        nc = plan.plane(plan.ncontrib, i).cpu().numpy()
        assert np.array_equal(nc[strict], o["n_contrib"][strict])


@pytest.mark.parametrize("tw", [8, 32])
def test_gradients_match_oracle_for_tile_shape(orc, tw):
    p, _, n, cams = _scene()
    cam = cams[0]
    plan = plan_for([cam], n_cap=p.shape[1], tile_w=tw)
    P = _dev(p)
    plan.render(P, n)
    o = orc.render(p, n, cam)
    rng = np.random.default_rng(tw)
    Wt = rng.uniform(-1, 1, (3, cam["height"], cam["width"])).astype(np.float32)
    Wt[:, o["amb"] != 0] = 0.0
    grad = torch.zeros_like(P)
    plan.backward(P, n, _dev(Wt).reshape(-1).contiguous(), grad)
    torch.cuda.synchronize()
    ref = orc.render_backward(p, n, cam, Wt)
    ids = np.nonzero(np.linalg.norm(ref[:, :n], axis=0) > 0)[0]
    check_gradients(grad.cpu().numpy().astype(np.float64), ref, ids, f"tile_w {tw}")


@pytest.mark.parametrize("tw", [8, 32])
def test_degenerate_scene_for_tile_shape(orc, tw):
    """The edge-case primitives (culled, near-plane, off-screen, huge, needle,
    faint, opaque, dark, tied) on the ragged 97x61 view with 8x32 and 32x8
    tiles: forward within the parity bar, gradients to the sampled bar."""
    from tests.gpu_util import compare_image

    p, cam, kinds = scenes.degenerate_scene(0)
    n = kinds.size
    plan = plan_for([cam], n_cap=p.shape[1], tile_w=tw)
    P = _dev(p)
    plan.render(P, n, with_ncontrib=True)
    torch.cuda.synchronize()
    assert not plan.overflowed()
    o = orc.render(p, n, cam)
    img = plan.image(plan.rgb, 0).cpu().numpy()
    T = plan.plane(plan.T, 0).cpu().numpy()
    m_img, m_T, n_amb, _, ok = compare_image(img, T, o)
    print(f"degenerate, tile_w {tw}: max|dI|={m_img:.2e} ambiguous={n_amb}/{ok.size}")
    assert m_img <= 1e-4 and m_T <= 1e-4
    strict = o["amb"] == 0
    nc = plan.plane(plan.ncontrib, 0).cpu().numpy()
    assert np.array_equal(nc[strict], o["n_contrib"][strict])
    rng = np.random.default_rng(tw)
    Wt = rng.uniform(-1, 1, (3, cam["height"], cam["width"])).astype(np.float32)
    Wt[:, o["amb"] != 0] = 0.0
    grad = torch.zeros_like(P)
    plan.backward(P, n, _dev(Wt).reshape(-1).contiguous(), grad)
    torch.cuda.synchronize()
    ref = orc.render_backward(p, n, cam, Wt)
    ids = np.nonzero(np.linalg.norm(ref[:, :n], axis=0) > 0)[0]
    # the degenerate scene's percentile bound (needle log-scales under random-sign weights)
    check_gradients(grad.cpu().numpy().astype(np.float64), ref, ids, f"degenerate tile_w {tw}", p99=0.3)
