"""Pins of the oracle's hand-derived reverse mode (the back-propagation of the Eq. 4
loss through Eq. 3 to position, rotation, scaling, density and SH, Section 3.3).

Two independent references:
* central finite differences in float64 (h = 1e-4) of <W, I> with W ~ U(-1, 1)
  per pixel and channel, skipping parameters whose +-h changes the set of
  composited Gaussians (a discrete event the derivative does not see);
* torch float64 autograd of a separate, vectorised re-implementation of the
  forward on tiny scenes.
"""

import numpy as np
import pytest
import torch

import scenes

ROWS = {"mean": slice(0, 3), "logscale": slice(3, 6), "quat": slice(6, 10), "opacity": slice(10, 11),
        "sh": slice(11, 59)}


def _tiny(seed, n=40, W=32, H=28, bg=(0.2, 0.5, 0.1), spread=0.35):
    rng = np.random.default_rng(seed)
    p = np.zeros((59, scenes.pad_cap(n)))
    p[0:3, :n] = np.stack([rng.uniform(-spread, spread, n), rng.uniform(-spread, spread, n),
                           rng.uniform(1.5, 2.5, n)])
    p[3:6, :n] = rng.normal(-2.7, 0.4, (3, n))
    p[6:10, :n] = rng.normal(size=(4, n))
    p[10, :n] = rng.normal(0.5, 1.2, n)
    p[11:14, :n] = rng.normal(0.3, 0.4, (3, n))
    p[14:59, :n] = rng.normal(0, 0.15, (45, n))
    ang = rng.normal(size=3) * 0.05
    c, s = np.cos(ang[1]), np.sin(ang[1])
    R = np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    cam = scenes.pinhole(W, H, 36.0, 38.0, W / 2 - 0.3, H / 2 + 0.2, R=R, t=[0.02, -0.01, 0.05], bg=bg)
    return p, cam


# ---------------------------------------------------------------------------
# torch float64 re-implementation (vectorised over pixels x Gaussians)
# ---------------------------------------------------------------------------
def _sh_torch(d):
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = np.pi
    k = [0.5 * np.sqrt(1 / pi), np.sqrt(3 / (4 * pi)), 0.5 * np.sqrt(15 / pi), 0.25 * np.sqrt(5 / pi),
         0.25 * np.sqrt(15 / pi), 0.25 * np.sqrt(35 / (2 * pi)), 0.5 * np.sqrt(105 / pi),
         0.25 * np.sqrt(21 / (2 * pi)), 0.25 * np.sqrt(7 / pi), 0.25 * np.sqrt(105 / pi)]
    one = torch.ones_like(x)
    return torch.stack([
        k[0] * one, -k[1] * y, k[1] * z, -k[1] * x,
        k[2] * x * y, -k[2] * y * z, k[3] * (2 * z * z - x * x - y * y), -k[2] * x * z,
        k[4] * (x * x - y * y),
        -k[5] * y * (3 * x * x - y * y), k[6] * x * y * z, -k[7] * y * (4 * z * z - x * x - y * y),
        k[8] * z * (2 * z * z - 3 * x * x - 3 * y * y), -k[7] * x * (4 * z * z - x * x - y * y),
        k[9] * z * (x * x - y * y), -k[5] * x * (x * x - 3 * y * y)], 1)


def torch_render(P, n, cam):
    """Differentiable float64 render of Eq. 3 (brute force over all pixel x Gaussian pairs)."""
    P = P[:, :n]
    Wm = torch.tensor(np.asarray(cam["R"], np.float64))
    t = torch.tensor(np.asarray(cam["t"], np.float64))
    fx, fy, cx, cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    Wd, Hd = cam["width"], cam["height"]
    mu = P[0:3].T
    s = torch.exp(P[3:6].T)
    q = P[6:10].T
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    Rq = torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)], 1)
    M = Rq * s[:, None, :]
    Sig = M @ M.transpose(1, 2)
    xc = mu @ Wm.T + t
    zc = xc[:, 2]
    assert bool((zc > 0.2).all())
    limx, limy = 1.3 * Wd / (2 * fx), 1.3 * Hd / (2 * fy)
    u = torch.clamp(xc[:, 0] / zc, -limx, limx)
    v = torch.clamp(xc[:, 1] / zc, -limy, limy)
    zero = torch.zeros_like(zc)
    J = torch.stack([torch.stack([fx / zc, zero, -fx * u / zc], 1),
                     torch.stack([zero, fy / zc, -fy * v / zc], 1)], 1)
    T2 = J @ Wm
    S2 = T2 @ Sig @ T2.transpose(1, 2) + 0.3 * torch.eye(2, dtype=torch.float64)
    det = S2[:, 0, 0] * S2[:, 1, 1] - S2[:, 0, 1] * S2[:, 1, 0]
    a = S2[:, 1, 1] / det
    b = -S2[:, 0, 1] / det
    c = S2[:, 0, 0] / det
    mx = fx * xc[:, 0] / zc + cx
    my = fy * xc[:, 1] / zc + cy
    o = torch.sigmoid(P[10])
    Cw = -(Wm.T @ t)
    dv = mu - Cw
    d = dv / dv.norm(dim=1, keepdim=True)
    Y = _sh_torch(d)                                   # [n,16]
    sh = P[11:59].T.reshape(n, 16, 3)
    rgb = torch.clamp_min(0.5 + (Y[:, :, None] * sh).sum(1), 0.0)
    order = torch.argsort(zc.detach(), stable=True)
    py, px = torch.meshgrid(torch.arange(Hd, dtype=torch.float64), torch.arange(Wd, dtype=torch.float64),
                            indexing="ij")
    px = px.reshape(-1, 1)
    py = py.reshape(-1, 1)
    dx = mx[order][None, :] - px
    dy = my[order][None, :] - py
    pw = -0.5 * (a[order] * dx * dx + c[order] * dy * dy) - b[order] * dx * dy
    at = o[order] * torch.exp(pw)
    contrib = (at >= 1 / 255).detach()
    alpha = torch.where(contrib, torch.clamp_max(at, 0.99), torch.zeros_like(at))
    om = 1 - alpha
    Tin = torch.cat([torch.ones_like(om[:, :1]), torch.cumprod(om, 1)[:, :-1]], 1)
    stop = (Tin * om < 1e-4).detach() & contrib
    stopped_before = torch.cumsum(stop.to(torch.int64), 1) > 0
    keep = contrib & ~stopped_before
    alpha = torch.where(keep, alpha, torch.zeros_like(alpha))
    om = 1 - alpha
    Tin = torch.cat([torch.ones_like(om[:, :1]), torch.cumprod(om, 1)[:, :-1]], 1)
    Tfin = Tin[:, -1] * om[:, -1]
    bg = torch.tensor(np.asarray(cam["bg"], np.float64))
    C = (alpha * Tin) @ rgb[order] + Tfin[:, None] * bg[None, :]
    return C.T.reshape(3, Hd, Wd), keep.sum(1).reshape(Hd, Wd)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_torch_forward_agrees(orc, seed):
    p, cam = _tiny(seed)
    n = 40
    img, nk = torch_render(torch.tensor(p), n, cam)
    r = orc.render(p, n, cam)
    np.testing.assert_allclose(r["img"], img.numpy(), atol=1e-12)
    assert np.array_equal(r["n_contrib"], nk.numpy())


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_backward_matches_torch_autograd(orc, seed):
    p, cam = _tiny(seed)
    n = 40
    rng = np.random.default_rng(50 + seed)
    Wt = rng.uniform(-1, 1, (3, cam["height"], cam["width"]))
    P = torch.tensor(p, requires_grad=True)
    img, _ = torch_render(P, n, cam)
    (img * torch.tensor(Wt)).sum().backward()
    ref = P.grad.numpy()[:, :n]
    got = orc.render_backward(p, n, cam, Wt)[:, :n]
    scale = np.abs(ref).max()
    np.testing.assert_allclose(got, ref, rtol=1e-8, atol=1e-10 * scale)


def test_backward_matches_torch_with_clamps(orc):
    """FOV clamp active (Gaussians outside the frustum whose splat still reaches the
    image), negative colours clamped, alpha clamped at 0.99, no dilation."""
    p, cam = _tiny(7, spread=1.0)
    n = 40
    p[10, :5] = 8.0                 # opacity ~1: alpha clamp 0.99
    p[11:14, 5:10] = -3.0           # colour clamp
    p[0, 10:13] = [1.6, -1.7, 1.9]  # far off-axis: FOV clamp (|u| > 1.3 * 32 / 72)
    p[3:6, 10:13] = -0.8            # large enough to reach into the image
    Wt = np.random.default_rng(3).uniform(-1, 1, (3, cam["height"], cam["width"]))
    rec = orc.preprocess(p, n, cam)
    u = (rec[:, 1] - cam["cx"]) / cam["fx"]
    assert (np.abs(u[10:13]) > 1.3 * cam["width"] / (2 * cam["fx"])).all()
    P = torch.tensor(p, requires_grad=True)
    img, _ = torch_render(P, n, cam)
    (img * torch.tensor(Wt)).sum().backward()
    ref = P.grad.numpy()[:, :n]
    got = orc.render_backward(p, n, cam, Wt)[:, :n]
    assert np.abs(ref[:, 10:13]).max() > 0       # the clamped Gaussians do reach pixels
    np.testing.assert_allclose(got, ref, rtol=1e-8, atol=1e-10 * np.abs(ref).max())


def _active_signature(orc, p, n, cam):
    r = orc.render(p, n, cam, prune=False)
    return r["n_contrib"], r["counts"]["contributing"]


def test_backward_matches_finite_differences(orc):
    p, cam = _tiny(11, n=30, W=24, H=24)
    n = 30
    rng = np.random.default_rng(1)
    Wt = rng.uniform(-1, 1, (3, 24, 24))
    g = orc.render_backward(p, n, cam, Wt)
    h = 1e-4
    comp = orc.render(p, n, cam)["n_contrib"]
    checked = 0
    worst = 0.0
    for gid in rng.permutation(n)[:10]:
        for name, rows in ROWS.items():
            fd, ref = [], []
            for r in range(rows.start, rows.stop):
                pp, pm = p.copy(), p.copy()
                pp[r, gid] += h
                pm[r, gid] -= h
                sp = _active_signature(orc, pp, n, cam)
                sm = _active_signature(orc, pm, n, cam)
                if not (np.array_equal(sp[0], sm[0]) and sp[1] == sm[1]):
                    continue
                Lp = (orc.render(pp, n, cam, prune=False)["img"] * Wt).sum()
                Lm = (orc.render(pm, n, cam, prune=False)["img"] * Wt).sum()
                fd.append((Lp - Lm) / (2 * h))
                ref.append(g[r, gid])
            if len(fd) == 0:
                continue
            fd, ref = np.array(fd), np.array(ref)
            denom = max(np.linalg.norm(fd), 1e-6)
            err = np.linalg.norm(fd - ref) / denom
            worst = max(worst, err)
            checked += 1
            assert err <= 1e-2, (gid, name, fd, ref)
    assert checked >= 30 and comp.max() > 2


def test_gradient_2d_zero_for_invisible(orc):
    p, cam = _tiny(2)
    p[0:3, 0] = [0, 0, -1.0]     # behind the camera
    Wt = np.ones((3, cam["height"], cam["width"]))
    g = orc.render_backward(p, 40, cam, Wt)
    assert np.all(g[:, 0] == 0)


def test_footprint_fd_equals_full_render_fd(orc):
    """The footprint-local finite difference equals the one from full re-renders."""
    p, cam = _tiny(5, n=30, W=24, H=24)
    n = 30
    Wt = np.random.default_rng(2).uniform(-1, 1, (3, 24, 24))
    rows = np.array([0, 2, 4, 7, 10, 11, 20, 58], np.int32)
    for gid in (3, 17):
        fd, changed = orc.fd_gauss(p, n, cam, Wt, gid, rows, h=1e-4)
        for k, r in enumerate(rows):
            pp, pm = p.copy(), p.copy()
            pp[r, gid] += 1e-4
            pm[r, gid] -= 1e-4
            ref = ((orc.render(pp, n, cam)["img"] - orc.render(pm, n, cam)["img"]) * Wt).sum() / 2e-4
            assert fd[k] == pytest.approx(ref, rel=1e-7, abs=1e-9)


def test_footprint_fd_is_thread_count_invariant_and_matches_analytic(orc):
    """On a saturated view (60,000 primitives, 160x96) the footprint finite
    difference differences each pixel before summing in pixel order: 1 and 8
    threads give the same bits, and it agrees with the analytic reverse mode
    to the 1e-2 relative bound of central differences (h = 1e-4)."""
    import scenes

    n = 60000
    p, _, cams = scenes.room_scene(4, n, 1, width=160, height=96, f=80.0)
    cam = cams[0]
    rng = np.random.default_rng(5)
    Wt = rng.uniform(-1, 1, (3, 96, 160))
    o = orc.render(p, n, cam)
    Wt[:, o["amb"] != 0] = 0.0
    g, g2d = orc.render_backward(p, n, cam, Wt, with_2d=True)
    seen = np.nonzero(np.abs(g2d[:, 6:9]).sum(axis=1) > 0)[0]
    ids = rng.choice(seen, 12, replace=False)
    rows = np.array(list(range(0, 11)) + [11, 12, 13, 20, 40], np.int32)
    before = orc.num_threads()
    try:
        orc.set_threads(1)
        fd1, ch1 = orc.fd_gauss(p, n, cam, Wt, ids, rows, h=1e-4)
        orc.set_threads(8)
        fd8, ch8 = orc.fd_gauss(p, n, cam, Wt, ids, rows, h=1e-4)
    finally:
        orc.set_threads(before)
    assert np.array_equal(fd1, fd8) and np.array_equal(ch1, ch8)
    checked = 0
    for a, gid in enumerate(ids):
        for name, rr in ROWS.items():
            sel = [i for i, r in enumerate(rows) if rr.start <= r < rr.stop and not ch1[a, i]]
            if not sel:
                continue
            f = fd1[a, sel]
            if np.linalg.norm(f) < 1e-8:
                continue
            e = np.linalg.norm(g[rows[sel], gid] - f) / np.linalg.norm(f)
            assert e <= 1e-2, (gid, name, e)
            checked += 1
    assert checked >= 20
