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


def test_online_step_at_rebound_level_matches_oracle():
    """One OnlineMapper step on keyframe k at the pyramid level Eq. 5 gives it,
    in a per-level plan whose view slot held another keyframe just before,
    against the FP64 oracle at that level's camera: the rendered image (max
    |diff| <= 1e-4 on pixels without an FP32-ambiguous decision), the Eq. 4
    loss against the oracle's pyramid of the keyframe image, the gradients of
    that loss on 64 sampled Gaussians (relative error <= 1e-3, same loss
    gradient on both sides, zero at flagged pixels) and the fused Adam update
    of the step.  Every input is seeded on the host: the map, the Adam moments
    and step, the keyframes' use counts, and ground-truth images rendered by
    the oracle from the perturbed map."""
    import oracle as orc
    import scenes
    from paper_2311_16728_amd.online import OnlineMapper
    from tests.gpu_util import check_gradients, compare_image, level_cam

    W, H, f, n, n_kf = 256, 192, 128.0, 30000, 3
    p, tp, cams = scenes.room_scene(17, n, n_kf, W, H, f)
    gt = [orc.render(tp, n, cam)["img"].astype(np.float32) for cam in cams]
    om = OnlineMapper(torch.as_tensor(p).cuda(), n, cams, [torch.as_tensor(g).cuda() for g in gt], levels=3, tau=2)
    mp = om.mapper
    rng = np.random.default_rng(23)
    m0 = np.zeros(p.shape, np.float32)
    v0 = np.zeros(p.shape, np.float32)
    m0[:, :n] = rng.normal(0.0, 1e-7, (59, n))
    v0[:, :n] = rng.uniform(0.0, 1e-13, (59, n))
    mp.m.copy_(torch.as_tensor(m0))
    mp.v.copy_(torch.as_tensor(v0))
    mp.step_count = 6
    k = 1
    om.schedule.uses = {0: 3, 1: 2, 2: 5}     # keyframe 1: its third use, level 2 - 2 // 2 = 1
    level = om.schedule.level(k)
    assert level == 1
    om.bind(level, 0).render(mp.params, n)      # the level's view slot held keyframe 0
    torch.cuda.synchronize()
    P0 = p.astype(np.float64)
    cam = level_cam(cams[k], level)
    gt_l = orc.pyramid(gt[k], 3)[level]
    o = orc.render(P0, n, cam)
    L, dI, _ = orc.loss(o["img"], gt_l, 0.2)
    print(f"keyframe {k} level {level} ({cam['width']}x{cam['height']}), oracle loss {L:.6f}", flush=True)

    # gradients of the same loss: the plan's unfused backward with the oracle's dL/dI
    plan = om.bind(level, k)
    plan.render(mp.params, n)
    dIz = dI.copy()
    dIz[:, o["amb"] != 0] = 0.0
    grad = torch.zeros_like(mp.params)
    plan.backward(mp.params, n, torch.as_tensor(dIz.astype(np.float32)).cuda().reshape(-1).contiguous(), grad)
    ref = orc.render_backward(P0, n, cam, dIz)
    g = grad.cpu().numpy().astype(np.float64)
    ids = np.nonzero(np.linalg.norm(ref[:, :n], axis=0) > 0)[0]
    assert len(ids) > 300
    check_gradients(g, ref, ids, f"online k={k} l={level}")

    # the online step itself: bind, render, loss, fused backward + Adam
    om.active = [k]
    om.step()
    torch.cuda.synchronize()
    assert om.log[-1] == (k, level) and mp.step_count == 7
    img = plan.image(plan.rgb, 0).cpu().numpy()
    e_img, e_T, n_amb, _, _ = compare_image(img, plan.plane(plan.T, 0).cpu().numpy(), o)
    print(f"image max|d| {e_img:.2e} T {e_T:.2e} flagged {n_amb}")
    assert e_img <= 1e-4 and e_T <= 1e-4 and n_amb <= 0.01 * cam["width"] * cam["height"]
    assert float(plan.d_total[0]) == pytest.approx(L, rel=1e-4)
    g_full = orc.render_backward(P0, n, cam, dI)
    pp, _, _ = orc.adam(P0, g_full, m0.astype(np.float64), v0.astype(np.float64), n,
                        mp.lr_rows.astype(np.float64), 7)
    got = mp.params.cpu().numpy().astype(np.float64)
    d_ref = pp[:, :n] - P0[:, :n]
    d_got = got[:, :n] - P0[:, :n]
    # updates whose gradient is clearly resolved move as the oracle's do
    rms = np.sqrt((g_full[:, :n] ** 2).mean(axis=1, keepdims=True))
    strong = np.abs(g_full[:, :n]) > 1e-3 * rms
    ok = np.abs(d_got - d_ref) <= 1e-3 * np.abs(d_ref) + 2e-7 * np.abs(P0[:, :n]) + 1e-9
    frac = ok[strong].mean()
    print(f"resolved updates matching: {frac:.4f} of {int(strong.sum())}")
    assert frac >= 0.995
