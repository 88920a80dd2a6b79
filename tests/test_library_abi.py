"""CPU checks of the C interface: the library loads and exports every entry point
that include/gs.h declares, host-only helpers behave, and invalid arguments
are rejected before any device work.  No kernel is launched."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2311_16728_amd", "libgs.so")
HEADER = os.path.join(ROOT, "include", "gs.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2311_16728_amd import build

        build.build()
    return C.CDLL(LIB)


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(gs_\w+)\s*\(", src, flags=re.M)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 12
    for nm in names:
        assert hasattr(lib, nm), nm


def test_binding_names_match_header():
    from paper_2311_16728_amd import gs

    assert sorted(gs.EXPORTED) == declared_functions()


def test_default_settings_and_status(lib):
    from paper_2311_16728_amd import gs

    s = gs.default_settings()
    assert s.alpha_min == pytest.approx(1 / 255) and s.alpha_max == pytest.approx(0.99)
    assert s.t_min == pytest.approx(1e-4) and s.sh_degree == 3 and s.batch == 256
    lib.gs_status_string.restype = C.c_char_p
    assert lib.gs_status_string(0) == b"ok"


def test_targets_layout_offsets():
    from paper_2311_16728_amd import gs
    import scenes

    cams = [scenes.pinhole(1200, 680, 600.0), scenes.pinhole(75, 33, 40.0)]
    views = [gs.make_view(c) for c in cams]
    specs = [(0, 0, (0, 0, 0), 1.0), (0, 1, (0, 0, 0), 1.0), (0, 2, (0, 0, 0), 1.0),
             (1, 0, (0, 0, 0), 1.0), (1, 1, (0, 0, 0), 1.0)]
    t, pix, tiles = gs.gs_targets_layout(views, specs)
    sizes = [(t[i].width, t[i].height) for i in range(5)]
    assert sizes == [(1200, 680), (600, 340), (300, 170), (75, 33), (38, 17)]
    exp_tiles = [75 * 43, 38 * 22, 19 * 11, 5 * 3, 3 * 2]
    assert [t[i].tiles_x * t[i].tiles_y for i in range(5)] == exp_tiles
    assert [t[i].tile_offset for i in range(5)] == list(np.cumsum([0] + exp_tiles[:-1]))
    assert [t[i].pix_offset for i in range(5)] == list(np.cumsum([0] + [w * h for w, h in sizes[:-1]]))
    assert pix == sum(w * h for w, h in sizes) and tiles == sum(exp_tiles)


def test_invalid_arguments_rejected():
    from paper_2311_16728_amd import gs
    import scenes

    views = [gs.make_view(scenes.pinhole(64, 64, 64.0))]
    with pytest.raises(gs.GsError):
        gs.gs_targets_layout(views, [(1, 0, (0, 0, 0), 1.0)])      # view out of range
    t, _, _ = gs.gs_targets_layout(views, [(0, 0, (0, 0, 0), 1.0)])
    s = gs.default_settings()
    with pytest.raises(gs.GsError):
        gs.gs_workspace_query(s, 100, 1, t, 1 << 10)                 # n_cap not a multiple of 64
    sizes = gs.gs_workspace_query(s, 256, 1, t, 1 << 10)
    assert sizes.proj_bytes >= 40 * 256 and sizes.accum_bytes >= 36 * 256
    # null device pointers fail validation on the host without touching a GPU
    lib = gs._lib
    assert lib.gs_preprocess(C.byref(s), None, 10, 256, None, 1, None, None) == 1
    assert lib.gs_adam_step(None, None, None, None, 10, 256, None, 0.9, 0.999, 1e-15, 1, None, None) == 1
    assert lib.gs_pyramid_build(None, 3, 10, 10, 3, None, None) == 1
    bad = gs.default_settings(batch=100)
    assert lib.gs_render_fwd(C.byref(bad), C.c_void_p(1), 256, 1, C.c_void_p(1), 1024, C.c_void_p(1),
                             1, 16, C.c_void_p(1), C.c_void_p(1), C.c_void_p(1), None, None, None) == 1
    rule = gs.densify_rule(5.0)
    one = C.c_void_p(16)
    assert lib.gs_densify(C.byref(rule), None, one, one, one, one, 10, 256, one, one, one, 256, one, one,
                          None) == 1
    assert lib.gs_densify(C.byref(rule), one, one, one, one, one, 10, 100, one, one, one, 256, one, one,
                          None) == 1                                # n_cap not a multiple of 64
    assert lib.gs_densify_stats(None, 10, 256, one, 1, one, None) == 1
    assert lib.gs_reset_opacity(one, None, None, 10, 256, 1.5, None) == 1
    assert gs.gs_densify_workspace_bytes(1 << 20) >= 16 * (1 << 10)


def test_binding_rejects_wrong_tensors():
    """The Python layer checks dtype, layout and shape before any device call."""
    import torch

    from paper_2311_16728_amd import gs

    s = gs.default_settings()
    bad_dtype = torch.zeros(59, 64, dtype=torch.float64)
    with pytest.raises(gs.GsError, match="float32"):
        gs.gs_preprocess(s, bad_dtype, 1, None, 1, None)
    bad_rows = torch.zeros(58, 64, dtype=torch.float32)
    with pytest.raises(gs.GsError, match="59 rows"):
        gs.gs_preprocess(s, bad_rows, 1, None, 1, None)
    not_contig = torch.zeros(64, 59, dtype=torch.float32).t()
    with pytest.raises(gs.GsError, match="contiguous"):
        gs.gs_preprocess(s, not_contig, 1, None, 1, None)
    on_host = torch.zeros(59, 64, dtype=torch.float32)
    with pytest.raises(gs.GsError, match="device"):
        gs.gs_preprocess(s, on_host, 1, None, 1, None)


def test_size_limits_rejected_on_the_host():
    """The size limits the header states are checked before anything is
    enqueued: pair capacity below 2^31 and (view, Gaussian) records below 2^32
    for binning, column capacities below 2^31 for densification, a tile grid
    that fits int32, tile widths 8 / 16 / 32 only, and column capacities that
    are multiples of 64 for the loop-closure correction."""
    from paper_2311_16728_amd import gs
    import scenes

    lib = gs._lib
    one = C.c_void_p(16)
    s = gs.default_settings()
    INVALID, CAPACITY = 1, 2
    # binning: pair_cap = 2^31, then 65 views x 2^26 columns (> 2^32 records)
    assert lib.gs_bin_sort(C.byref(s), one, 10, 256, 1, one, 1, 16, one, 1 << 31, one, None) == INVALID
    assert lib.gs_bin_sort(C.byref(s), one, 10, 1 << 26, 65, one, 1, 16, one, 1 << 20, one, None) == INVALID
    # densification: input or output capacity 2^31
    rule = gs.densify_rule(5.0)
    assert lib.gs_densify(C.byref(rule), one, one, one, one, one, 10, 1 << 31, one, one, one, 256, one, one,
                          None) == INVALID
    assert lib.gs_densify(C.byref(rule), one, one, one, one, one, 10, 256, one, one, one, 1 << 31, one, one,
                          None) == INVALID
    assert lib.gs_densify(C.byref(rule), one, one, one, one, one, 10, 256, one, one, one, 100, one, one,
                          None) == INVALID                          # out_cap not a multiple of 64
    # densification without a workspace: above its fixed scratch (n > 2^24) it
    # reports the capacity; invalid arguments as gs_densify
    big_n = gs.DENSIFY_NOALLOC_MAX_N + 1
    assert lib.gs_densify_noalloc(C.byref(rule), one, one, one, one, one, big_n, big_n + 63, one, one, one,
                                  256, one, None) == CAPACITY
    assert lib.gs_densify_noalloc(C.byref(rule), one, one, one, one, one, 10, 256, one, one, one, 100, one,
                                  None) == INVALID
    assert lib.gs_densify_noalloc(C.byref(rule), one, one, one, one, one, 10, 256, one, one, one, 256, None,
                                  None) == INVALID
    # loop closure: n_cap not a multiple of 64, no transform
    assert lib.gs_sim3_apply(one, 10, 100, one, 1, None, one, None) == INVALID
    assert lib.gs_sim3_apply(one, 10, 256, one, 0, None, one, None) == INVALID
    # tile grid: 2^30 x 2^30 pixels in 16 x 16 tiles overflow int32 tile indices
    big = [gs.make_view(scenes.pinhole(1 << 30, 1 << 30, 1000.0))]
    vbig = (gs.gs_view * 1)(*big)
    tg = (gs.gs_target * 1)()
    tg[0].view, tg[0].level, tg[0].tile_w = 0, 0, 16
    tot_p, tot_t = C.c_int64(), C.c_int32()
    assert lib.gs_targets_layout(vbig, 1, tg, 1, C.byref(tot_p), C.byref(tot_t)) == CAPACITY
    # tile widths other than 8 / 16 / 32
    small = (gs.gs_view * 1)(gs.make_view(scenes.pinhole(64, 64, 64.0)))
    for w, want in ((12, INVALID), (64, INVALID), (8, 0), (32, 0)):
        tg[0].tile_w = w
        assert lib.gs_targets_layout(small, 1, tg, 1, C.byref(tot_p), C.byref(tot_t)) == want, w


def test_checked_mode_and_status_word():
    """Checked mode needs a status word; the status word maps to the status codes
    the header states; record counts past 2^32 - 1 are refused by every call that
    indexes projection records."""
    from paper_2311_16728_amd import gs

    lib = gs._lib
    one = C.c_void_p(16)
    INVALID = 1
    s = gs.default_settings()
    assert s.checked == 0 and not s.status
    no_word = gs.default_settings(checked=1)
    assert lib.gs_preprocess(C.byref(no_word), one, 10, 256, one, 1, one, None) == INVALID
    with_word = gs.default_settings(checked=1, status=16)
    views = [gs.make_view(__import__("scenes").pinhole(64, 64, 64.0))]
    t, _, _ = gs.gs_targets_layout(views, [(0, 0, (0, 0, 0), 1.0)])
    gs.gs_workspace_query(with_word, 256, 1, t, 1 << 10)
    with pytest.raises(gs.GsError):
        gs.gs_workspace_query(no_word, 256, 1, t, 1 << 10)
    assert gs.gs_status_word(0) == 0
    assert gs.gs_status_word(gs.STATUS_PAIR_OVERFLOW) == 2          # capacity
    assert gs.gs_status_word(gs.STATUS_NUMERIC) == 5                # numeric
    assert gs.gs_status_word(gs.STATUS_NUMERIC | gs.STATUS_PAIR_OVERFLOW) == 5
    assert gs.gs_status_word(8) == INVALID
    lib.gs_status_string.restype = C.c_char_p
    assert lib.gs_status_string(5) == b"non-finite value"
    with pytest.raises(gs.GsError, match="capacity"):
        gs.check_status_word(gs.STATUS_PAIR_OVERFLOW)
    # 65 views x 2^26 columns: more than 2^32 - 1 records
    nv, ncap = 65, 1 << 26
    assert lib.gs_preprocess(C.byref(s), one, 10, ncap, one, nv, one, None) == INVALID
    assert lib.gs_render_fwd(C.byref(s), one, ncap, nv, one, 1024, one, 1, 16, one, one, one,
                             None, None, None) == INVALID
    assert lib.gs_raster_bwd(C.byref(s), one, ncap, nv, one, 1024, one, 1, 16, one, one, one, one,
                             None) == INVALID
    assert lib.gs_render_fwd(C.byref(s), one, 256, 1, one, 1 << 31, one, 1, 16, one, one, one,
                             None, None, None) == INVALID
    with pytest.raises(gs.GsError):
        gs.gs_workspace_query(s, ncap, nv, t, 1 << 10)
    with pytest.raises(gs.GsError):
        gs.gs_workspace_query(s, 256, 1, t, 1 << 31)
