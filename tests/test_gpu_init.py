"""GPU tests of the initialiser kernels against CPU references: the MLP against
float64 torch with the same BF16 roundings (BF16 x BF16 products are exact in
FP32, so only summation order and rare BF16 rounding flips of hidden units
differ), the 3-NN heuristic against scipy's KD-tree, feature extraction and
decoding against numpy/scipy."""

import numpy as np
import pytest
import torch
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import scenes
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

NW, NB = 38912, 272


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


def bf(t):
    """Round to BF16 (nearest even) and back to float64."""
    return torch.as_tensor(t).to(torch.float32).to(torch.bfloat16).to(torch.float64)


def unpack(w):
    w = torch.as_tensor(w, dtype=torch.float64)
    return w[:20480].view(128, 160), w[20480:36864].view(128, 128), w[36864:].view(16, 128)


def ref_forward(w, b, x):
    W1, W2, W3 = unpack(w)
    b = torch.as_tensor(b, dtype=torch.float64)
    h1 = bf(torch.relu(x @ W1.T + b[:128]))
    h2 = bf(torch.relu(h1 @ W2.T + b[128:256]))
    return h2 @ W3.T + b[256:], h1, h2


def _model(seed):
    rng = np.random.default_rng(seed)
    w = (rng.normal(size=NW) * np.concatenate([np.full(20480, 1 / np.sqrt(160)), np.full(16384, 1 / np.sqrt(128)),
                                              np.full(2048, 1 / np.sqrt(128))])).astype(np.float32)
    b = (rng.normal(size=NB) * 0.1).astype(np.float32)
    wb = bf(w)                                   # BF16 weights as float64
    return w, b, wb


@pytest.mark.parametrize("B", [4096, 100, 4133])
def test_mlp_forward(B):
    from paper_2311_16728_amd import gs

    w, b, wb = _model(B)
    rng = np.random.default_rng(1)
    x = bf(rng.normal(size=(B, 160)))
    x[:, 159:] = 0
    Wd = wb.to(torch.float32).to(torch.bfloat16).view(torch.int16).cuda()
    Xd = x.to(torch.float32).to(torch.bfloat16).view(torch.int16).cuda().contiguous()
    y = torch.zeros(B, 16, dtype=torch.float32, device="cuda")
    act = torch.zeros(2 * B * 128, dtype=torch.int16, device="cuda")
    gs.gs_init_mlp_fwd(Wd, torch.as_tensor(b).cuda(), Xd, y, act)
    torch.cuda.synchronize()
    ref, h1, _ = ref_forward(wb, b, x)
    scale = ref.abs().max().item()
    err = (y.cpu().double() - ref).abs().max().item()
    print(f"B={B}: mlp forward max |dy| {err:.2e} (scale {scale:.2f})")
    assert err <= 2e-3 * scale
    # hidden activations stored for the backward: all but rare BF16 rounding flips equal
    g1 = act[:B * 128].view(B, 128).view(torch.bfloat16).cpu().double()
    assert (g1 == h1).double().mean().item() >= 0.999


def _fp32_bound(absum, k):
    """Rigorous bound on the FP32 accumulation error of a length-k dot product
    of exact BF16 products plus a bias, in any summation order, doubled."""
    return 2.0 * (k + 1) * 2.0 ** -24 * absum


def _unambiguous_batch(wb, b, B, rng):
    """Inputs x (BF16) and upstream gradients dy whose hidden ReLU masks FP32
    decides as float64 does: rows with a pre-activation whose sign FP32 could
    decide differently are redrawn.  For the second layer that includes the
    effect of first-layer BF16 roundings FP32 could take the other way (each
    such hidden value may move by its rounding step).  A flipped mask moves a
    whole hidden gradient, about 5e-3 of the weight gradient's norm per flip;
    a BF16 rounding flip of one hidden value moves one product by one BF16 ulp
    and is left in."""
    W1, W2, W3 = unpack(wb)
    bb = torch.as_tensor(b, dtype=torch.float64)
    x = bf(rng.normal(size=(B, 160)))
    dy = torch.as_tensor(rng.normal(size=(B, 16)), dtype=torch.float64)
    for _ in range(100):
        p1 = x @ W1.T + bb[:128]
        d1 = _fp32_bound(x.abs() @ W1.abs().T + bb[:128].abs(), 160)
        ok = (p1.abs() > d1).all(1)
        h1 = bf(torch.relu(p1))
        step = (bf(torch.relu(p1 + d1)) - bf(torch.relu(p1 - d1))).abs()
        p2 = h1 @ W2.T + bb[128:256]
        d2 = _fp32_bound(h1.abs() @ W2.abs().T + bb[128:256].abs(), 128) + step @ W2.abs().T
        ok &= (p2.abs() > d2).all(1)
        bad = (~ok).nonzero().flatten()
        if bad.numel() == 0:
            return x, dy
        x[bad] = bf(rng.normal(size=(bad.numel(), 160)))
    raise AssertionError("could not draw an unambiguous batch")


def test_mlp_backward():
    from paper_2311_16728_amd import gs

    B = 2048
    w, b, wb = _model(7)
    rng = np.random.default_rng(2)
    x, dy = _unambiguous_batch(wb, b, B, rng)
    Wd = wb.to(torch.float32).to(torch.bfloat16).view(torch.int16).cuda()
    Xd = x.to(torch.float32).to(torch.bfloat16).view(torch.int16).cuda().contiguous()
    y = torch.zeros(B, 16, dtype=torch.float32, device="cuda")
    act = torch.zeros(2 * B * 128, dtype=torch.int16, device="cuda")
    bd = torch.as_tensor(b).cuda()
    gs.gs_init_mlp_fwd(Wd, bd, Xd, y, act)
    dw = torch.zeros(NW, dtype=torch.float32, device="cuda")
    db = torch.zeros(NB, dtype=torch.float32, device="cuda")
    gs.gs_init_mlp_bwd(Wd, Xd, act, dy.to(torch.float32).cuda(), dw, db)
    torch.cuda.synchronize()
    # reference with the same BF16 roundings, hidden activations recomputed in
    # float64 from the inputs (nothing read back from the kernel's workspace);
    # the inputs were drawn so that FP32 takes every ReLU mask decision the
    # same way
    W1, W2, W3 = unpack(wb)
    _, h1, h2 = ref_forward(wb, b, x)
    dyb = bf(dy)
    d2 = (dyb @ W3) * (h2 > 0)
    d2b = bf(d2)
    d1 = (d2b @ W2) * (h1 > 0)
    d1b = bf(d1)
    ref_w = torch.cat([(d1b.T @ x).reshape(-1), (d2b.T @ h1).reshape(-1), (dyb.T @ h2).reshape(-1)])
    ref_b = torch.cat([d1.sum(0), d2.sum(0), dy.sum(0)])
    gw, gb = dw.cpu().double(), db.cpu().double()
    for name, g, r, sl in [("W1", gw, ref_w, slice(0, 20480)), ("W2", gw, ref_w, slice(20480, 36864)),
                           ("W3", gw, ref_w, slice(36864, NW)), ("b", gb, ref_b, slice(0, NB))]:
        err = (g[sl] - r[sl]).norm().item() / r[sl].norm().item()
        print(f"mlp backward {name}: rel {err:.2e}")
        assert err <= 2e-3, name


def test_mlp_adam_and_training_reduces_loss():
    """A few hundred steps of the project's fwd/bwd/Adam fit a fixed random
    linear target: the loss drops by an order of magnitude."""
    from paper_2311_16728_amd.init_mlp import InitMLP

    rng = np.random.default_rng(3)
    B = 1024
    x = rng.normal(size=(B, 159)).astype(np.float32)
    A = (rng.normal(size=(159, 11)) / np.sqrt(159)).astype(np.float32)
    t = x @ A
    net = InitMLP(seed=0)
    xd = net.pack_inputs(torch.as_tensor(x).cuda())
    td = torch.as_tensor(t).cuda()
    first = net.train_step(xd, td, lr=3e-3)
    for _ in range(300):
        last = net.train_step(xd, td, lr=3e-3)
    print(f"training loss {first:.4f} -> {last:.4f}")
    assert last < 0.1 * first


def test_features_exact():
    from paper_2311_16728_amd import gs

    rng = np.random.default_rng(4)
    H, W, B = 37, 53, 300
    img = rng.uniform(size=(3, H, W)).astype(np.float32)
    kp = np.stack([rng.uniform(-2, W + 2, B), rng.uniform(-2, H + 2, B), rng.uniform(0.5, 5, B),
                   1.2 ** rng.integers(0, 9, B)], 1).astype(np.float32)
    heur = rng.normal(-3, 1, size=(59, B)).astype(np.float32)
    x = torch.zeros(B, 160, dtype=torch.int16, device="cuda")
    gs.gs_init_features(torch.as_tensor(img).cuda(), torch.as_tensor(kp).cuda(), x, torch.as_tensor(heur).cuda())
    torch.cuda.synchronize()
    got = x.view(torch.bfloat16).cpu().to(torch.float32).numpy()
    ref = np.zeros((B, 160), np.float32)
    for i in range(B):
        cu, cv = int(np.rint(kp[i, 0])), int(np.rint(kp[i, 1]))
        ys = np.clip(np.arange(cv - 3, cv + 4), 0, H - 1)
        xs = np.clip(np.arange(cu - 3, cu + 4), 0, W - 1)
        ref[i, :147] = img[:, ys][:, :, xs].reshape(-1)
        ref[i, 147] = kp[i, 2]
        ref[i, 148] = kp[i, 3]
        ref[i, 149 + min(max(int(np.rint(np.log(max(kp[i, 3], 1.0)) / np.log(1.2))), 0), 7)] = 1.0
        ref[i, 157] = heur[3, i]
        ref[i, 158] = np.log(kp[i, 2])
    ref = torch.as_tensor(ref).to(torch.bfloat16).to(torch.float32).numpy()
    # the octave and log depth use single-precision logs: allow BF16 rounding-boundary flips
    assert (got[:, :157] == ref[:, :157]).all(axis=1).mean() >= 0.99
    np.testing.assert_array_equal(got[:, 157], ref[:, 157])
    np.testing.assert_allclose(got[:, 158], ref[:, 158], rtol=1e-2, atol=1e-2)
    assert np.all(got[:, 159] == 0)


def test_heuristic_matches_kdtree():
    from paper_2311_16728_amd import gs

    rng = np.random.default_rng(5)
    n, ncap, B = 20000, 20480, 700
    p = np.zeros((59, ncap), np.float32)
    p[0:3, :n] = rng.uniform(-2, 2, (3, n))
    new = rng.uniform(-2, 2, (3, B)).astype(np.float32)
    rgb = rng.uniform(size=(3, B)).astype(np.float32)
    out = torch.zeros(59, B, dtype=torch.float32, device="cuda")
    gs.gs_init_heuristic(torch.as_tensor(new).cuda(), torch.as_tensor(rgb).cuda(),
                         torch.as_tensor(p).cuda(), n, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    allpts = np.concatenate([p[0:3, :n].T, new.T]).astype(np.float64)
    d, _ = cKDTree(allpts).query(new.T.astype(np.float64), k=4)   # first hit is the point itself
    ls = np.log(d[:, 1:4].mean(axis=1))
    np.testing.assert_allclose(o[3], ls, rtol=0, atol=2e-5)
    np.testing.assert_allclose(o[4], ls, atol=2e-5)
    np.testing.assert_allclose(o[0:3], new, rtol=0, atol=0)
    assert np.all(o[6] == 1) and np.all(o[7:10] == 0)
    np.testing.assert_allclose(o[10], np.log(0.1 / 0.9), rtol=1e-6)
    np.testing.assert_allclose(o[11:14], (rgb - 0.5) / (0.5 / np.sqrt(np.pi)), rtol=1e-5, atol=1e-6)
    assert np.all(o[14:] == 0)


def test_decode_and_append():
    from paper_2311_16728_amd import gs

    rng = np.random.default_rng(6)
    B = 500
    cam = scenes.pinhole(640, 480, 320.0, R=Rotation.from_rotvec([0.2, -0.4, 0.1]).as_matrix(),
                         t=[0.3, -0.1, 0.5])
    view = gs.make_view(cam)
    kp = np.stack([rng.uniform(0, 640, B), rng.uniform(0, 480, B), rng.uniform(0.5, 4, B),
                   np.ones(B)], 1).astype(np.float32)
    y = rng.normal(size=(B, 16)).astype(np.float32)
    y[:50, 7] = -8.0                     # predicted opacity < 0.01: heuristic fallback
    heur = rng.normal(size=(59, B)).astype(np.float32)
    out = torch.zeros(59, B, dtype=torch.float32, device="cuda")
    used = torch.zeros(B, dtype=torch.int32, device="cuda")
    gs.gs_init_decode(torch.as_tensor(y).cuda(), torch.as_tensor(kp).cuda(), view,
                      torch.as_tensor(heur).cuda(), out, used)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    u = used.cpu().numpy()
    assert np.all(u[:50] == 1) and np.all(u[50:] == 0)
    assert np.array_equal(o[:, :50], heur[:, :50])
    R = np.asarray(cam["R"], np.float64)
    t = np.asarray(cam["t"], np.float64)
    xc = np.stack([kp[:, 2] * (kp[:, 0] - cam["cx"]) / cam["fx"], kp[:, 2] * (kp[:, 1] - cam["cy"]) / cam["fy"],
                   kp[:, 2]], 1)
    mu = (xc - t) @ R
    np.testing.assert_allclose(o[0:3, 50:], mu[50:].T, rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(o[3:6, 50:], heur[3:6, 50:] + y[50:, 0:3].T, atol=1e-5)
    qc = y[50:, 3:7]
    rot_c = Rotation.from_quat(qc[:, [1, 2, 3, 0]])           # scipy: scalar last
    rot_w = Rotation.from_matrix(R.T) * rot_c
    qw = o[6:10, 50:].T
    got = Rotation.from_quat(qw[:, [1, 2, 3, 0]])
    np.testing.assert_allclose(got.as_matrix(), rot_w.as_matrix(), atol=2e-5)
    np.testing.assert_allclose(np.linalg.norm(qw, axis=1), np.linalg.norm(qc, axis=1), rtol=1e-5)
    np.testing.assert_allclose(o[10, 50:], y[50:, 7])
    np.testing.assert_allclose(o[11:14, 50:], heur[11:14, 50:] + y[50:, 8:11].T, atol=1e-6)
    assert np.all(o[14:, 50:] == 0)
    # append
    P = torch.ones(59, 1024, dtype=torch.float32, device="cuda")
    m = torch.ones_like(P)
    v = torch.ones_like(P)
    gs.gs_append(P, m, v, 300, out)
    torch.cuda.synchronize()
    assert torch.equal(P[:, 300:800], out)
    assert torch.all(m[:, 300:800] == 0) and torch.all(m[:, :300] == 1) and torch.all(m[:, 800:] == 1)


@pytest.mark.timeout(900)
def test_learned_initialiser_beats_heuristic():
    """Small version of the initialiser experiment: train on mapper-generated
    pairs from 6 seeded scenes (200k Gaussians, 4 keyframes), then on 6 unseen
    scenes start batched mapping from the heuristic and from the network.  The
    network predicts corrections to the heuristic, so on held-out pairs its
    log-scale and opacity errors must be below the heuristic's.  The
    photometric losses of both starts, before and after 100 mapping
    iterations, are printed, not asserted: with 6 training scenes they differ
    by less than the scene-to-scene spread (6 unseen scenes: final-loss gain
    -0.0005 +- 0.0032, the learned start lower in 2 of 6 before mapping); the
    loss comparison is measured at the experiment's size (20 training scenes,
    5 held-out) by the initialiser pipeline."""
    from paper_2311_16728_amd import init_pipeline as ip

    kw = dict(n=200_000, n_kf=4, per_kf=1024, kf_stride=1, min_weight=1.0)
    X, Y, H = ip.generate(range(6), 100, log=None, **kw)
    val = torch.arange(X.shape[0], device=X.device) % 10 == 0
    net, first, last = ip.train(X[~val].contiguous(), Y[~val].contiguous(), 1500, log=None)
    assert last < first
    pred = net.forward(X[val].contiguous())[:, :ip.N_TARGET]
    e_net, e_heur = ip.param_errors(pred, Y[val]), ip.param_errors(H[val], Y[val])
    print("parameter mse: learned", e_net, "heuristic", e_heur)
    assert e_net["log_scale"] < e_heur["log_scale"]
    assert e_net["opacity_logit"] < e_heur["opacity_logit"]
    res = ip.evaluate(net, range(1000, 1006), 100, log=None, **kw)
    print({k: v for k, v in res.items() if k != "rows"})
    init = [(r["learned"]["loss_init"], r["heuristic"]["loss_init"]) for r in res["rows"]]
    print("starting loss learned / heuristic:", init)
    assert res["scenes"] == 6 and all(np.isfinite(v) for pair in init for v in pair)
