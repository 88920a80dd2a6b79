"""Host-side logic that needs no GPU: the benchmark's single-GPU contract, the
batched workload's target layout, and the initialiser pipeline's quaternion
helpers."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_batched_workload_layout():
    from paper_2311_16728_amd import gs

    cams = scenes.mixed_keyframes(0, 32)
    sizes = sorted({(c["width"], c["height"]) for c in cams})
    assert sizes == [(640, 480), (752, 480), (1200, 680)]
    counts = {s: sum((c["width"], c["height"]) == s for c in cams) for s in sizes}
    assert counts == {(640, 480): 12, (752, 480): 10, (1200, 680): 10}
    views = [gs.make_view(c) for c in cams]
    specs = [(v, l, (0, 0, 0), 1.0) for v in range(32) for l in range(3)]
    targets, pixels, tiles = gs.gs_targets_layout(views, specs)
    assert len(targets) == 96
    expect_px, expect_tiles = 0, 0
    for c in cams:
        w, h = c["width"], c["height"]
        for _ in range(3):
            expect_px += w * h
            expect_tiles += ((w + 15) // 16) * ((h + 15) // 16)
            w, h = (w + 1) // 2, (h + 1) // 2
    assert pixels == expect_px and tiles == expect_tiles


def test_quaternion_helpers_match_scipy():
    from paper_2311_16728_amd.init_pipeline import _mat_to_quat, _quat_mul

    rng = np.random.default_rng(0)
    a = Rotation.random(50, random_state=1)
    b = Rotation.random(50, random_state=2)
    qa = torch.as_tensor(a.as_quat()[:, [3, 0, 1, 2]])
    qb = torch.as_tensor(b.as_quat()[:, [3, 0, 1, 2]])
    qc = _quat_mul(qa, qb).numpy()
    got = Rotation.from_quat(qc[:, [1, 2, 3, 0]]).as_matrix()
    np.testing.assert_allclose(got, (a * b).as_matrix(), atol=1e-12)
    R = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    q = _mat_to_quat(R)
    np.testing.assert_allclose(Rotation.from_quat(q[[1, 2, 3, 0]]).as_matrix(), R, atol=1e-12)


def test_mapping_learning_rates():
    from paper_2311_16728_amd.mapper import mapping_lr_rows

    lr = mapping_lr_rows(5.0)
    assert lr.shape == (59,) and lr.dtype == np.float32
    assert np.all(lr > 0)
    assert lr[10] > lr[3] > lr[11] > lr[14]


def test_pyramid_schedule_coarse_to_fine():
    """Eq. 5: level n first, one level finer every tau uses, then level 0 for good;
    keyframes are counted separately."""
    from paper_2311_16728_amd.mapper import PyramidSchedule

    sch = PyramidSchedule(levels=3, tau=4)
    seq = [sch.use("a") for _ in range(14)]
    assert seq == [2] * 4 + [1] * 4 + [0] * 6
    assert sch.use("b") == 2 and sch.level("a") == 0
    one = PyramidSchedule(levels=1, tau=2)
    assert [one.use(0) for _ in range(3)] == [0, 0, 0]
    with pytest.raises(ValueError):
        PyramidSchedule(levels=0)


def test_auto_backward_waves_by_tile_count():
    """Plans that leave the backward's waves per tile open get one wave from
    1,536 tiles on, two from 512, else four (the three pyramid levels of a
    1200x680 keyframe: 3,225 / 836 / 209 tiles)."""
    from paper_2311_16728_amd.mapper import auto_bwd_waves

    assert [auto_bwd_waves(t) for t in (3225, 836, 209)] == [1, 2, 4]
    assert [auto_bwd_waves(t) for t in (1536, 1535, 512, 511, 1)] == [1, 2, 2, 4, 4]


def test_tile_shapes_in_layout():
    from paper_2311_16728_amd import gs

    views = [gs.make_view(scenes.pinhole(150, 110, 100.0))]
    for tw, tx, ty in [(8, 19, 4), (16, 10, 7), (32, 5, 14)]:
        t, pix, tiles = gs.gs_targets_layout(views, [(0, 0, (0, 0, 0), 1.0)], tw)
        assert (t[0].tile_w, t[0].tiles_x, t[0].tiles_y, tiles, pix) == (tw, tx, ty, tx * ty, 150 * 110)
    t, _, _ = gs.gs_targets_layout(views, [(0, 0, (0, 0, 0), 1.0)], 0)
    assert t[0].tile_w == 16
    with pytest.raises(gs.GsError):
        gs.gs_targets_layout(views, [(0, 0, (0, 0, 0), 1.0)], 12)
    with pytest.raises(gs.GsError):
        gs.gs_targets_layout(views, [(0, 0, (0, 0, 0), 1.0)], 64)


def test_cpu_baseline_reports_threads_model_and_single_thread_rate():
    """The oracle baseline of the benchmark line names the CPU and reports a
    one-thread rate beside the all-threads one (tiny scene, whole image)."""
    sys.path.insert(0, ROOT)
    import bench
    import oracle

    p, _, cam = scenes.tiny_scene(0, n=300)
    target = np.zeros((3, cam["height"], cam["width"]))
    threads = oracle.num_threads()
    out = bench.cpu_baseline(p, 300, [cam], target, 1.0)
    assert oracle.num_threads() == threads   # restored after the one-thread run
    assert out["kind"] == "oracle" and out["cores"] == threads and out["value"] > 0
    assert isinstance(out["cpu_model"], str) and out["cpu_model"]
    st = out["single_thread"]
    assert st["cores"] == 1 and st["value"] > 0 and st["unit"] == "iters/s"
