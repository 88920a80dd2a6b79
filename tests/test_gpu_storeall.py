"""GPU checks of the store-all rasteriser variant (gs_render_fwd_store,
gs_raster_bwd_stored), the comparison point of the recompute backward
(back-propagation of Eq. 3, Section 3.3): its forward renders exactly what
gs_render_fwd renders; the stored transmittances lie in the stored layout
(non-increasing per pixel, within [1e-4, 1]); the backward from the store
matches the FP64 oracle with the gradient metric of the parity tests and the
recompute backward to FP32 rounding; a store that is too small is reported
and read by nothing."""

import numpy as np
import pytest
import torch

import scenes
from tests.gpu_util import check_gradients, plan_for, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def _cases():
    p, _, cam = scenes.tiny_scene(0)
    yield "tiny", p, 2000, cam
    p2, cam2, kinds = scenes.degenerate_scene(0)
    yield "degenerate", p2, kinds.size, cam2


def _store_run(plan, cap=None):
    from paper_2311_16728_amd import gs

    T = plan.total_tiles
    steps = torch.zeros(T, dtype=torch.int32, device="cuda")
    base = torch.zeros(T + 1, dtype=torch.int64, device="cuda")
    rgb, Tf = torch.empty_like(plan.rgb), torch.empty_like(plan.T)
    last, nc = torch.empty_like(plan.last), torch.empty_like(plan.ncontrib)
    # sizing call with an empty store, then the store at the reported size
    store = torch.zeros(1, dtype=torch.float32, device="cuda")
    args = (plan.settings, plan.proj_ws, plan.n_cap, plan.n_views, plan.sort_ws, plan.pair_cap,
            plan.targets_dev, plan.n_targets, T)
    gs.gs_render_fwd_store(*args, rgb, Tf, last, nc, steps, base, store)
    torch.cuda.synchronize()
    need = int(base[T].item())
    store = torch.full((need if cap is None else cap,), -1.0, dtype=torch.float32, device="cuda")
    gs.gs_render_fwd_store(*args, rgb, Tf, last, nc, steps, base, store)
    torch.cuda.synchronize()
    return dict(rgb=rgb, T=Tf, last=last, nc=nc, steps=steps, base=base, store=store, need=need)


@pytest.mark.parametrize("case", ["tiny", "degenerate"])
def test_store_forward_and_layout(case):
    name, p, n, cam = [c for c in _cases() if c[0] == case][0]
    plan = plan_for([cam], n_cap=p.shape[1])
    P = _dev(p)
    plan.render(P, n, with_ncontrib=True)
    r = _store_run(plan)
    torch.cuda.synchronize()
    assert torch.equal(r["rgb"], plan.rgb) and torch.equal(r["T"], plan.T)
    assert torch.equal(r["last"], plan.last) and torch.equal(r["nc"], plan.ncontrib)
    # layout: per tile 256 floats per step of its deepest pixel, tiles in order
    base = r["base"].cpu().numpy()
    steps = r["steps"].cpu().numpy()
    assert np.array_equal(np.diff(base), 256 * steps.astype(np.int64))
    nc = plan.plane(plan.ncontrib, 0).cpu().numpy()
    H, W = nc.shape
    store = r["store"].cpu().numpy()
    tw, th = 16, 16
    tx = (W + tw - 1) // tw
    for tile in range(plan.total_tiles):
        y0, x0 = (tile // tx) * th, (tile % tx) * tw
        blk = nc[y0:y0 + th, x0:x0 + tw]
        assert steps[tile] == (blk.max() if blk.size else 0)
    # every pixel: its stored transmittances are non-increasing in [1e-4, 1],
    # start at 1 and stop above the final transmittance
    Tfin = plan.plane(plan.T, 0).cpu().numpy()
    for y in range(0, H, 7):
        for x in range(0, W, 5):
            k = nc[y, x]
            if k == 0:
                continue
            tile = (y // th) * tx + x // tw
            lp = (y % th) * tw + (x % tw)
            seq = store[base[tile] + 256 * np.arange(k) + lp]
            assert seq[0] == 1.0 and np.all(np.diff(seq) <= 0) and seq.min() >= 1e-4
            assert seq[-1] >= Tfin[y, x]


@pytest.mark.parametrize("case", ["tiny", "degenerate"])
def test_stored_backward_matches_oracle_and_recompute(orc, case):
    from paper_2311_16728_amd import gs

    name, p, n, cam = [c for c in _cases() if c[0] == case][0]
    plan = plan_for([cam], n_cap=p.shape[1])
    P = _dev(p)
    plan.render(P, n, with_ncontrib=True)
    o = orc.render(p, n, cam)
    rng = np.random.default_rng(11)
    Wt = rng.uniform(-1, 1, (3, cam["height"], cam["width"])).astype(np.float32)
    Wt[:, o["amb"] != 0] = 0.0
    dL = _dev(Wt).reshape(-1).contiguous()
    # recompute backward
    grad_r = torch.zeros_like(P)
    plan.backward(P, n, dL, grad_r)
    acc_r = plan.accum_ws.clone()
    # store-all backward
    r = _store_run(plan)
    gs.gs_raster_bwd_stored(plan.settings, plan.proj_ws, plan.n_cap, plan.n_views, plan.sort_ws, plan.pair_cap,
                            plan.targets_dev, plan.n_targets, plan.total_tiles, r["last"], r["nc"], r["base"],
                            r["store"], dL, plan.accum_ws)
    grad_s = torch.zeros_like(P)
    gs.gs_project_bwd(plan.settings, P, n, plan.views_dev, plan.n_views, plan.accum_ws, grad_s)
    torch.cuda.synchronize()
    a_r = acc_r.view(torch.float32)[: 9 * n].cpu().numpy().reshape(n, 9)
    a_s = plan.accum_ws.view(torch.float32)[: 9 * n].cpu().numpy().reshape(n, 9)
    scale = np.abs(a_r).max(axis=0) + 1e-30
    print(case, "stored vs recompute accumulators, max rel to column max:", (np.abs(a_s - a_r) / scale).max())
    assert (np.abs(a_s - a_r) / scale).max() <= 1e-4
    g = grad_s.cpu().numpy().astype(np.float64)
    ref = orc.render_backward(p, n, cam, Wt)
    ids = np.nonzero(np.linalg.norm(ref[:, :n], axis=0) > 0)[0]
    check_gradients(g, ref, ids, case + " stored", p99=0.1 if case == "tiny" else 0.3)


def test_store_too_small_is_reported_and_not_read():
    from paper_2311_16728_amd import gs

    name, p, n, cam = list(_cases())[0]
    plan = plan_for([cam], n_cap=p.shape[1])
    P = _dev(p)
    plan.render(P, n, with_ncontrib=True)
    full = _store_run(plan)
    short = _store_run(plan, cap=full["need"] - 1)
    assert short["need"] == full["need"] and int(short["base"][-1].item()) > short["store"].numel()
    assert torch.all(short["store"] == -1.0)          # nothing stored
    assert torch.equal(short["rgb"], plan.rgb)         # the image is still rendered
    dL = torch.ones(3 * plan.total_pixels, dtype=torch.float32, device="cuda")
    plan.accum_ws.fill_(7)
    gs.gs_raster_bwd_stored(plan.settings, plan.proj_ws, plan.n_cap, plan.n_views, plan.sort_ws, plan.pair_cap,
                            plan.targets_dev, plan.n_targets, plan.total_tiles, short["last"], short["nc"],
                            short["base"], short["store"], dL, plan.accum_ws)
    torch.cuda.synchronize()
    acc = plan.accum_ws.view(torch.float32)[: 9 * plan.n_views * plan.n_cap]
    assert torch.all(acc == 0)
