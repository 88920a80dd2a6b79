"""Online mapping with per-keyframe pyramid levels (Section 3.4, Eq. 5): the
schedule each keyframe follows, the view binding of the shared per-level
plans, and that the online run improves the map."""

import numpy as np
import pytest
import torch

from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def scene():
    from paper_2311_16728_amd.online import online_scene

    return online_scene(5, n_gt=40000, n_kf=4, width=320, height=240, f=160.0, per_kf=500)


def test_online_schedule_binding_and_progress(scene):
    from paper_2311_16728_amd.mapper import RenderPlan
    from paper_2311_16728_amd.online import OnlineMapper, run_online

    # before any training: the initial map's PSNR
    om0 = OnlineMapper(scene["params"].clone(), scene["n"], scene["cams"], scene["gt_images"], levels=3)
    om0.active = list(range(4))
    psnr0 = om0.psnr()
    r = run_online(scene, levels=3, tau=4, geo=True, iters=240, join_every=20, densify_every=50)
    om = r["mapper"]
    print({k: v for k, v in r.items() if k != "mapper"}, "initial PSNR", psnr0)
    # Eq. 5 per keyframe: level 2 for its first 4 uses, level 1 for the next 4, then level 0
    for k in range(4):
        levels = [l for (kk, l) in om.log if kk == k]
        expect = [max(0, 2 - i // 4) for i in range(len(levels))]
        assert levels == expect and len(levels) > 12
    # keyframes join in order, one every 20 iterations
    first = {}
    for i, (k, _) in enumerate(om.log):
        first.setdefault(k, i)
    assert all(first[k] >= 20 * k for k in range(4))
    # the shared plan bound to keyframe k at level l renders what a plan of its own renders
    P, n = om.mapper.params, om.mapper.n
    for k, l in [(3, 0), (1, 2), (2, 1)]:
        plan = om.bind(l, k)
        plan.render(P, n)
        own = RenderPlan([scene["cams"][k]], [(0, l, (0.0, 0.0, 0.0), 1.0)], P.shape[1], 1 << 26)
        own.render(P, n)
        torch.cuda.synchronize()
        assert torch.equal(plan.rgb, own.rgb)
    # geometry-based densification added every keyframe's keypoints, and training helped
    assert r["primitives"] != scene["n"]
    assert r["psnr"] > psnr0 + 1.0
