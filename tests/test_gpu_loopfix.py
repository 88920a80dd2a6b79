"""GPU parity of the loop-closure correction (gs_sim3_apply) against the FP64
oracle, and its render invariance.

Bars: centres within 1e-5 (coordinates up to ~15 m), log-scales and
quaternions within 1e-6, SH coefficients within 2e-6 (the band matrices are
built in float32 from a collocation whose condition numbers stay below 4),
opacity and untouched primitives bit-exact; a moved map rendered from the
correspondingly moved camera within 1e-4 of the oracle's render of the
original (pixels without FP32-ambiguous compositing decisions).
"""

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import scenes
from oracle import loopfix as lf
from tests.gpu_util import compare_image, plan_for, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _sims(seed, k):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        q = Rotation.random(random_state=seed * 100 + i).as_quat()[[3, 0, 1, 2]]
        q = q * rng.uniform(0.5, 2.0)          # the library normalises
        out.append((q.astype(np.float32), rng.normal(0, 1.0, 3).astype(np.float32),
                    np.float32(np.exp(rng.normal(0, 0.3)))))
    return out


def _apply_gpu(p, n, sims, assign=None):
    from paper_2311_16728_amd import gs

    P = _dev(p)
    xf = gs.sim3_table(sims)
    ws = torch.empty(gs.gs_sim3_workspace_bytes(len(sims)), dtype=torch.uint8, device="cuda")
    gs.gs_sim3_apply(P, n, xf, len(sims), ws, None if assign is None else _dev(assign))
    torch.cuda.synchronize()
    return P.cpu().numpy()


def _check(got, ref, p, cols, moved):
    g, r = got[:, cols].astype(np.float64), ref[:, cols]
    mv = moved[cols]
    assert np.abs(g[0:3] - r[0:3]).max() <= 1e-5
    assert np.abs(g[3:10] - r[3:10]).max() <= 1e-6
    assert np.array_equal(got[10, cols], p[10, cols])
    assert np.abs(g[11:59] - r[11:59]).max() <= 2e-6
    # untouched primitives are bit-exact
    assert np.array_equal(got[:, cols][:, ~mv], p[:, cols][:, ~mv])


@pytest.mark.parametrize("n", [1, 300, 3001])
def test_sim3_matches_oracle(n):
    c = scenes.densify_case(11, n)
    p = c["params"]
    sims = _sims(1, 4) + [((0.0, 0.0, 0.0, 0.0), (1.0, 0.0, 0.0), 1.0),   # zero quaternion: invalid
                          ((1.0, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0), 0.0)]   # s = 0: invalid
    rng = np.random.default_rng(n)
    assign = rng.integers(-1, 8, size=n).astype(np.int32)   # -1, 6 and 7 are out of range
    got = _apply_gpu(p, n, sims, assign)
    ref = lf.apply_sim3(p, n, sims[:4], assign)   # indices 4, 5 are invalid transforms: unchanged
    moved = (assign >= 0) & (assign < 4)
    _check(got, ref, p, np.arange(n), moved)
    assert np.array_equal(got[:, n:], p[:, n:])


def test_sim3_single_transform_and_identity():
    c = scenes.densify_case(12, 2000)
    p = c["params"]
    sims = _sims(2, 1)
    got = _apply_gpu(p, 2000, sims)
    ref = lf.apply_sim3(p, 2000, sims)
    _check(got, ref, p, np.arange(2000), np.ones(2000, bool))
    ident = _apply_gpu(p, 2000, [((1, 0, 0, 0), (0, 0, 0), 1.0)])
    assert np.abs(ident[:, :2000] - p[:, :2000]).max() <= 1e-6
    assert np.array_equal(ident[0:11], p[0:11])


def test_sim3_full_size_sampled():
    """One million primitives, 128 keyframe corrections, 2000 sampled columns."""
    rng = np.random.default_rng(3)
    p = scenes.draw_gaussians(rng, 1_000_000, scenes.ROOM_LO, scenes.ROOM_HI)
    sims = _sims(3, 128)
    assign = rng.integers(0, 128, size=1_000_000).astype(np.int32)
    got = _apply_gpu(p, 1_000_000, sims, assign)
    cols = np.unique(np.r_[rng.integers(0, 1_000_000, 2000), 0, 999_999])
    sub = np.ascontiguousarray(p[:, cols])
    ref = np.zeros_like(p, dtype=np.float64)
    ref[:, cols] = lf.apply_sim3(sub, len(cols), sims, assign[cols])[:, :len(cols)]
    _check(got, ref, p, cols, np.ones(1_000_000, bool))


@pytest.mark.parametrize("scale", [1.0, 1.6])
def test_moved_map_renders_like_moved_camera(orc, scale):
    p, _, cam = scenes.tiny_scene(4, n=1500)
    q = Rotation.from_rotvec([-0.4, 0.7, 0.2]).as_quat()[[3, 0, 1, 2]]
    sim = (q.astype(np.float32), np.array([0.7, 0.3, -2.0], np.float32), np.float32(scale))
    moved = _apply_gpu(p, 1500, [sim])
    cam2 = lf.moved_camera(cam, sim)
    cam2["R"] = np.asarray(cam2["R"], np.float32)
    cam2["t"] = np.asarray(cam2["t"], np.float32)
    plan = plan_for([cam2], n_cap=p.shape[1])
    plan.render(_dev(moved), 1500)
    torch.cuda.synchronize()
    img = plan.image(plan.rgb, 0).cpu().numpy()
    T = plan.plane(plan.T, 0).cpu().numpy()
    o = orc.render(p, 1500, cam)
    m_img, m_T, n_amb, _, ok = compare_image(img, T, o)
    print(f"scale {scale}: max|dI|={m_img:.2e} max|dT|={m_T:.2e} ambiguous={n_amb}")
    assert m_img <= 1e-4 and m_T <= 1e-4
