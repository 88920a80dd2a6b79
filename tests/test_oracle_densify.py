"""Pins of the densification oracle (Section 3.3.1, the split / clone / prune
rule of 3D Gaussian splatting) against hand-derived outcomes, a closed-form
statistic, the law of the split children's centres and invariants."""

import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenes
from oracle import densify as od

EXTENT = 10.0   # log_dense = ln 0.1, log_big = ln 1 = 0


def _hand_case():
    n_cap = 64
    P = np.zeros((59, n_cap), np.float32)
    stats = np.zeros((2, n_cap), np.float32)
    noise = np.zeros((6, n_cap), np.float32)
    P[6, :9] = 1.0                                   # identity rotation unless set below
    P[11:59, :9] = np.arange(48)[:, None] * 0.01 + np.arange(9)[None, :]
    rows = [  # log-scales, logit, (grad sum, visits)
        ((-3, -3, -3), 0.0, (1e-4, 1)),      # 0 below threshold: kept
        ((-3, -3.5, -4), 1.0, (9e-4, 3)),    # 1 mean 3e-4, small: cloned
        ((-1, -2, -2.5), 0.5, (5e-4, 1)),    # 2 large: split
        ((-3, -3, -3), -6.0, (0, 0)),        # 3 faint: pruned
        ((0.5, -3, -3), 2.0, (0, 2)),        # 4 too big in the world: pruned
        ((-2, -2, -2), 0.0, (0, 0)),         # 5 never visited: kept
        ((-4, -4, -4), -7.0, (1e-3, 1)),     # 6 cloned but faint: original and copy pruned
        ((-0.5, -3, -3), 0.0, (3e-4, 1)),    # 7 split, rotated 90 degrees about z
        ((0.6, -1, -1), 0.0, (1e-3, 1)),     # 8 split, children still too big: none kept
    ]
    for g, (ls, lo, st) in enumerate(rows):
        P[0:3, g] = (g, 2 * g, -g)
        P[3:6, g] = ls
        P[10, g] = lo
        stats[:, g] = st
    P[6:10, 7] = (math.cos(math.pi / 4), 0, 0, math.sin(math.pi / 4))
    noise[0:3, 2] = (1, 0, 0)
    noise[3:6, 2] = (0, -1, 0)
    noise[0:3, 7] = (1, 0, 0)
    noise[3:6, 7] = (0, 0, 2)
    m = np.random.default_rng(0).normal(size=(59, n_cap)).astype(np.float32)
    v = np.abs(np.random.default_rng(1).normal(size=(59, n_cap))).astype(np.float32)
    return P, m, v, stats, noise


def test_hand_built_outcomes():
    P, m, v, stats, noise = _hand_case()
    out, om, ov, counts = od.densify(P, m, v, stats, 9, noise, od.densify_rule(EXTENT))
    assert counts == dict(n_out=8, cloned=1, split=3, pruned=3)
    # survivors in order, then the copy of 1, the children of 2 and of 7
    src = [0, 1, 5, 1, 2, 2, 7, 7]
    for j, g in enumerate(src):
        np.testing.assert_array_equal(out[6:, j], P[6:, g].astype(np.float64))
    np.testing.assert_array_equal(out[:, :4], P[:, [0, 1, 5, 1]].astype(np.float64))
    sh = math.log(1.6)
    mu2, mu7 = P[0:3, 2].astype(np.float64), P[0:3, 7].astype(np.float64)
    np.testing.assert_allclose(out[0:3, 4], mu2 + (math.exp(-1), 0, 0), atol=1e-12)
    np.testing.assert_allclose(out[0:3, 5], mu2 + (0, -math.exp(-2), 0), atol=1e-12)
    np.testing.assert_allclose(out[0:3, 6], mu7 + (0, math.exp(-0.5), 0), atol=1e-7)
    np.testing.assert_allclose(out[0:3, 7], mu7 + (0, 0, 2 * math.exp(-3)), atol=1e-7)
    np.testing.assert_allclose(out[3:6, 4], np.array([-1, -2, -2.5]) - sh, atol=1e-12)
    np.testing.assert_allclose(out[3:6, 6], np.array([-0.5, -3, -3]) - sh, atol=1e-12)
    # moments: survivors keep theirs, new primitives start from zero
    np.testing.assert_array_equal(om[:, :3], m[:, [0, 1, 5]].astype(np.float64))
    np.testing.assert_array_equal(ov[:, :3], v[:, [0, 1, 5]].astype(np.float64))
    assert not om[:, 3:].any() and not ov[:, 3:].any()


def test_no_size_pruning_when_disabled():
    P, m, v, stats, noise = _hand_case()
    _, _, _, counts = od.densify(P, m, v, stats, 9, noise, od.densify_rule(EXTENT, big_fraction=None))
    # 4 survives, and 8's children survive
    assert counts == dict(n_out=11, cloned=1, split=3, pruned=2)


def test_split_children_sample_the_parent_gaussian():
    """Children centres are draws from N(mu, R S^2 R^T): their sample
    covariance approaches the covariance built by scipy's rotation."""
    rng = np.random.default_rng(5)
    n = 20000
    P = np.zeros((59, n), np.float32)
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    ls = np.array([-0.7, -1.6, -2.4])
    P[3:6] = ls[:, None]
    P[6:10] = q[:, None]
    stats = np.zeros((2, n), np.float32)
    stats[:] = 1.0
    noise = rng.normal(size=(6, n)).astype(np.float32)
    out, _, _, counts = od.densify(P, P, P, stats, n, noise, od.densify_rule(EXTENT, big_fraction=None))
    assert counts["split"] == n and counts["n_out"] == 2 * n
    off = out[0:3].T
    q, ls = P[6:10, 0].astype(np.float64), P[3:6, 0].astype(np.float64)   # as stored
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    cov = R @ np.diag(np.exp(2 * ls)) @ R.T
    emp = off.T @ off / off.shape[0]
    assert np.linalg.norm(emp - cov) < 0.03 * np.linalg.norm(cov)
    # the offsets are R (s * z) exactly, column by column
    z = noise.astype(np.float64)
    s = np.exp(ls)
    np.testing.assert_allclose(out[0:3, 0::2], R @ (s[:, None] * z[0:3]), atol=1e-9)
    np.testing.assert_allclose(out[0:3, 1::2], R @ (s[:, None] * z[3:6]), atol=1e-9)


def test_statistic_closed_form():
    acc = np.zeros((2, 3, 9))
    acc[0, 0, :2] = (3e-6, -4e-6)
    acc[0, 0, 5] = 1.0                 # other values do not enter the norm
    acc[1, 1, 7] = 2e-3                # colour only: a visit with a zero norm
    st = od.densify_stats(acc, [(1200, 680), (640, 480)])
    expect0 = math.hypot(3e-6 * 600, 4e-6 * 340)
    np.testing.assert_allclose(st[:, 0], (expect0, 1.0), rtol=1e-15)
    np.testing.assert_array_equal(st[:, 1], (0.0, 1.0))
    np.testing.assert_array_equal(st[:, 2], (0.0, 0.0))
    st2 = od.densify_stats(acc, [(1200, 680), (640, 480)], st)
    np.testing.assert_allclose(st2, 2 * st)


def test_random_case_invariants():
    c = scenes.densify_case(3, 3000)
    rule = od.densify_rule(c["extent"])
    n = c["n"]
    action, keep, new = od.decide(c["params"], c["stats"], n, rule)
    out, om, ov, counts = od.densify(c["params"], c["m"], c["v"], c["stats"], n, c["noise"], rule)
    K = int(keep.sum())
    assert counts["n_out"] == K + int(new.sum()) == out.shape[1]
    assert counts["pruned"] == n - counts["split"] - K
    assert 0 < counts["cloned"] and 0 < counts["split"] and 0 < counts["pruned"]
    P = c["params"].astype(np.float64)
    np.testing.assert_array_equal(out[:, :K], P[:, np.nonzero(keep)[0]])
    assert not om[:, K:].any() and not ov[:, K:].any()
    # every new column is a copy of its parent or a child of it
    j = K
    for g in np.nonzero(new)[0]:
        for _ in range(new[g]):
            np.testing.assert_array_equal(out[6:, j], P[6:, g])
            if action[g] == od.CLONE:
                np.testing.assert_array_equal(out[:6, j], P[:6, g])
            else:
                np.testing.assert_allclose(out[3:6, j], P[3:6, g] - math.log(1.6), atol=1e-12)
            j += 1
    # nothing that survives breaks the pruning rule
    ls32 = out[3:6].astype(np.float32).max(axis=0)
    assert np.all(out[10].astype(np.float32) >= rule["logit_min"])
    assert np.all(ls32 <= rule["log_big"] + 1e-6)


def test_reset_opacity_closed_form():
    P = np.zeros((59, 64), np.float32)
    P[10, :4] = (-6.0, -4.0, 0.0, 3.0)
    m = np.ones((59, 64), np.float32)
    out, om, ov = od.reset_opacity(P, m, m, 4)
    cap = math.log(0.01 / 0.99)
    np.testing.assert_allclose(out[10, :4], (-6.0, cap, cap, cap), atol=1e-6)
    assert not om[10, :4].any() and om[10, 4:].all() and om[9].all() and ov[11].all()


def test_library_rule_matches_oracle_rule():
    """The library's host-side rule builder rounds the same thresholds."""
    from paper_2311_16728_amd import gs

    for extent, kw in [(10.0, {}), (3.7, dict(grad_threshold=5e-4, percent_dense=0.02)),
                       (0.5, dict(min_opacity=0.01, big_fraction=None))]:
        a = gs.densify_rule(extent, **kw)
        b = od.densify_rule(extent, **kw)
        for k in ("grad_threshold", "log_dense", "log_big", "logit_min", "log_shrink"):
            assert np.float32(getattr(a, k)) == b[k], k
    with pytest.raises(gs.GsError):
        gs.densify_rule(-1.0)
