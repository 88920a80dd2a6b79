"""GPU tests of batching: all (keyframe, level) targets in one launch equal the
per-target renders bitwise; pyramid levels match the oracle rendering at the
level's intrinsics; a captured HIP graph replays the eager iteration."""

import numpy as np
import pytest
import torch

import scenes
from tests.gpu_util import compare_image, plan_for, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _two_views():
    p, _, cam = scenes.tiny_scene(9, n=1500)
    c2 = scenes.pinhole(150, 110, 130.0, 125.0, 71.3, 52.6,
                        R=[[0.995, 0, 0.0998], [0, 1, 0], [-0.0998, 0, 0.995]], t=[0.1, 0.0, 0.1],
                        bg=(0.1, 0.2, 0.3))
    return p, 1500, [cam, c2]


def test_batched_equals_per_target_bitwise():
    p, n, cams = _two_views()
    P = _dev(p)
    big = plan_for(cams, levels=(0, 1, 2), n_cap=p.shape[1])
    big.render(P, n)
    torch.cuda.synchronize()
    k = 0
    for v, cam in enumerate(cams):
        for l in range(3):
            one = plan_for([cam], levels=(l,), n_cap=p.shape[1])
            one.render(P, n)
            torch.cuda.synchronize()
            assert torch.equal(one.image(one.rgb, 0), big.image(big.rgb, k))
            assert torch.equal(one.plane(one.T, 0), big.plane(big.T, k))
            k += 1


def test_pyramid_levels_match_oracle(orc):
    p, n, cams = _two_views()
    plan = plan_for(cams, levels=(0, 1, 2), n_cap=p.shape[1])
    plan.render(_dev(p), n)
    torch.cuda.synchronize()
    k = 0
    for cam in cams:
        for l in range(3):
            lc = scenes.level_camera(cam, l)
            o = orc.render(p, n, lc)
            img = plan.image(plan.rgb, k).cpu().numpy()
            T = plan.plane(plan.T, k).cpu().numpy()
            m_img, m_T, n_amb, _, ok = compare_image(img, T, o)
            assert m_img <= 1e-4 and m_T <= 1e-4, (k, m_img, m_T)
            k += 1


def test_batched_gradients_match_oracle(orc):
    """Backward over all levels of two views: the per-(view, Gaussian)
    accumulators sum level contributions in level-0 units."""
    from tests.gpu_util import check_gradients

    p, n, cams = _two_views()
    plan = plan_for(cams, levels=(0, 1, 2), n_cap=p.shape[1])
    P = _dev(p)
    plan.render(P, n)
    rng = np.random.default_rng(3)
    W = np.zeros(3 * plan.total_pixels, np.float32)
    ref = np.zeros((59, p.shape[1]))
    k = 0
    for cam in cams:
        for l in range(3):
            lc = scenes.level_camera(cam, l)
            o = orc.render(p, n, lc)
            Wt = rng.uniform(-1, 1, (3, lc["height"], lc["width"]))
            Wt[:, o["amb"] != 0] = 0.0
            off, w, h = plan.target_slice(k)
            W[3 * off:3 * (off + w * h)] = Wt.astype(np.float32).reshape(-1)
            ref += orc.render_backward(p, n, lc, Wt)
            k += 1
    grad = torch.zeros_like(P)
    plan.backward(P, n, _dev(W), grad)
    g = grad.cpu().numpy().astype(np.float64)
    ids = np.nonzero(np.linalg.norm(ref[:, :n], axis=0) > 0)[0]
    check_gradients(g, ref, ids, "batched")


def test_graph_replay_matches_eager():
    """Three replays of a captured iteration, with eager work and synchronisation
    between them, equal three eager iterations from the same state."""
    from paper_2311_16728_amd.batching import BatchedMapper
    from paper_2311_16728_amd.mapper import RenderPlan

    p, n, cams = _two_views()
    _, tp, _ = scenes.tiny_scene(9, n=1500)
    gts = []
    for cam in cams:
        pl = RenderPlan([cam], [(0, 0, (0, 0, 0), 1.0)], p.shape[1], 1 << 20)
        pl.render(_dev(tp), n)
        gts.append(pl.image(pl.rgb, 0).clone())
    eager = BatchedMapper(_dev(p), n, cams, gts, pair_cap=1 << 20)
    graphed = BatchedMapper(_dev(p), n, cams, gts, pair_cap=1 << 20)
    # the graphed mapper's warm-up iteration is matched by one eager iteration
    eager.iteration()
    graphed.capture(warmup=1)
    torch.cuda.synchronize()
    for r in range(3):
        eager.iteration()
        graphed.step()
        torch.cuda.synchronize()
        _ = (graphed.params.sum() + 1).item()     # unrelated eager work between replays
        assert graphed.step_count == eager.step_count == r + 2
        scale = eager.params.abs().max(dim=1, keepdim=True).values + 1e-30
        diff = ((graphed.params - eager.params).abs() / scale).max().item()
        assert diff <= 1e-5, (r, diff)
        assert torch.equal(graphed.plan.rgb, eager.plan.rgb) or \
            (graphed.plan.rgb - eager.plan.rgb).abs().max().item() <= 1e-5


def test_wide_tile_sort_equals_per_target():
    """22 keyframes at 1200x680 hold 70,950 tiles (17-bit tile keys, sorted with
    two 9-bit passes); every target equals its own single-target render (12-bit
    keys, two 8-bit passes) bitwise."""
    p, _, cams = scenes.room_scene(5, 50_000, n_keyframes=22)
    n = 50_000
    P = _dev(p)
    big = plan_for(cams, levels=(0,), n_cap=p.shape[1], pair_cap=1 << 24)
    assert big.total_tiles > 1 << 16
    big.render(P, n)
    torch.cuda.synchronize()
    assert not big.overflowed()
    for v in (0, 7, 21):
        one = plan_for([cams[v]], levels=(0,), n_cap=p.shape[1], pair_cap=1 << 22)
        one.render(P, n)
        torch.cuda.synchronize()
        assert torch.equal(one.image(one.rgb, 0), big.image(big.rgb, v)), v
        assert torch.equal(one.plane(one.T, 0), big.plane(big.T, v)), v


def test_group_scan_path_equals_per_target_bitwise():
    """Two room views of 600k Gaussians: 4,688 count workgroups, more than the
    compaction sums by itself (4,096), so the two-view binning scans the
    workgroup counts first, while each view alone (2,344 workgroups) takes the
    self-summing path.  Images and transmittance agree bitwise."""
    n = 600_000
    p, _, cams = scenes.room_scene(3, n, n_keyframes=2, width=320, height=180, f=160.0)
    P = _dev(p)
    big = plan_for(cams, n_cap=p.shape[1], pair_cap=1 << 23)
    assert big.n_views * ((big.n_cap + 255) // 256) > 4096
    big.render(P, n)
    torch.cuda.synchronize()
    assert not big.overflowed()
    for v, cam in enumerate(cams):
        one = plan_for([cam], n_cap=p.shape[1], pair_cap=1 << 23)
        one.render(P, n)
        torch.cuda.synchronize()
        assert not one.overflowed()
        assert torch.equal(one.image(one.rgb, 0), big.image(big.rgb, v)), v
        assert torch.equal(one.plane(one.T, 0), big.plane(big.T, v)), v
    assert float(big.rgb.abs().sum()) > 0


def test_many_targets_equal_per_target_bitwise():
    """400 views x 3 levels = 1,200 targets: more views and listed targets than
    the binning keeps in LDS (256) and more targets than one staging pass of
    the per-view lists (1,024).  Sampled targets, among them ones beyond both
    limits, render bitwise as they do alone."""
    p, _, _ = scenes.tiny_scene(7, n=2000)
    n = 2000
    rng = np.random.default_rng(5)
    cams = [scenes.pinhole(40, 24, 30.0, t=rng.uniform(-0.3, 0.3, 3)) for _ in range(400)]
    P = _dev(p)
    big = plan_for(cams, levels=(0, 1, 2), n_cap=p.shape[1], pair_cap=1 << 23)
    assert big.n_targets == 1200
    big.render(P, n)
    torch.cuda.synchronize()
    assert not big.overflowed()
    for k in (0, 1, 255, 256, 257, 767, 1023, 1024, 1025, 1100, 1198, 1199):
        v, l = divmod(k, 3)
        one = plan_for([cams[v]], levels=(l,), n_cap=p.shape[1])
        one.render(P, n)
        torch.cuda.synchronize()
        assert torch.equal(one.image(one.rgb, 0), big.image(big.rgb, k)), k
        assert torch.equal(one.plane(one.T, 0), big.plane(big.T, k)), k
    # the renders are not all background
    assert float(big.rgb.abs().sum()) > 0


@pytest.mark.parametrize("waves", [1, 2, 4])
def test_queue_schedule_matches_grid(waves):
    """Persistent raster workgroups over the cost-ordered tile queue (schedule
    1: forward and backward; 2: backward only) render bitwise what one
    workgroup per tile renders, on every launch in a row (the queue resets
    itself), and their gradients agree to FP32 summation order."""
    from paper_2311_16728_amd import gs

    p, n, cams = _two_views()
    P = _dev(p)
    rng = np.random.default_rng(5)
    out = {}
    for sched in (0, 1, 2):
        s = gs.default_settings(batch=128, bwd_waves=waves, schedule=sched)
        plan = plan_for(cams, levels=(0, 1, 2), n_cap=p.shape[1], settings=s)
        W = _dev(rng.uniform(-1, 1, 3 * plan.total_pixels).astype(np.float32)) if sched == 0 else out[0][4]
        runs = []
        for rep in range(3):   # the second and third launches reuse the reset queue
            plan.preprocess(P, n)
            plan.bin_sort(n)
            for _ in range(2):   # two forwards on one binning
                plan.render_fwd()
            grad = torch.zeros_like(P)
            plan.backward(P, n, W, grad)
            torch.cuda.synchronize()
            runs.append((plan.rgb.clone(), plan.T.clone(), plan.last.clone(), grad.cpu().numpy()))
        for r in runs[1:]:
            assert torch.equal(r[0], runs[0][0]) and torch.equal(r[2], runs[0][2])
        out[sched] = runs[0] + (W,) if sched == 0 else runs[0]
    r0, t0, l0, g0, _ = out[0]
    scale = np.abs(g0).max(axis=1, keepdims=True) + 1e-30
    for sched in (1, 2):
        r1, t1, l1, g1 = out[sched]
        assert torch.equal(r0, r1) and torch.equal(t0, t1) and torch.equal(l0, l1)
        assert (np.abs(g1 - g0) / scale).max() <= 1e-5
