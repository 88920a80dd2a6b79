"""ctypes binding of libgs (the C interface in include/gs.h).

Argument marshalling only: every function here forwards torch device
pointers and the current HIP stream to the same-named C entry point and turns
a non-zero status into an exception.  All arithmetic runs in the HIP kernels;
if libgs.so is missing the import of this module fails.
"""

from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")

NUM_ROWS = 59
TILE = 16
STATUS_PAIR_OVERFLOW = 1
STATUS_NUMERIC = 2


class GsError(RuntimeError):
    pass


class gs_settings(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("znear", C.c_float), ("dilation", C.c_float), ("fov_clamp", C.c_float),
                ("sh_degree", C.c_int32), ("batch", C.c_int32), ("bwd_waves", C.c_int32),
                ("checked", C.c_int32), ("schedule", C.c_int32), ("status", C.c_void_p)]


class gs_view(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class gs_target(C.Structure):
    _fields_ = [("view", C.c_int32), ("level", C.c_int32), ("width", C.c_int32),
                ("height", C.c_int32), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("tile_offset", C.c_int32), ("tile_w", C.c_int32), ("pix_offset", C.c_int64),
                ("bg", C.c_float * 3), ("weight", C.c_float)]


class gs_densify_rule(C.Structure):
    _fields_ = [("grad_threshold", C.c_float), ("log_dense", C.c_float), ("log_big", C.c_float),
                ("logit_min", C.c_float), ("log_shrink", C.c_float)]


class gs_sim3(C.Structure):
    _fields_ = [("q", C.c_float * 4), ("t", C.c_float * 3), ("s", C.c_float)]


class gs_sizes(C.Structure):
    _fields_ = [("proj_bytes", C.c_size_t), ("sort_bytes", C.c_size_t),
                ("accum_bytes", C.c_size_t), ("loss_bytes", C.c_size_t)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2311_16728_amd.build.build() first")
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, f32 = C.c_void_p, C.c_int64, C.c_int32, C.c_float
    S, V, T = C.POINTER(gs_settings), C.POINTER(gs_view), C.POINTER(gs_target)
    sig = {
        "gs_status_string": ([C.c_int], C.c_char_p),
        "gs_status_word": ([C.c_uint32], C.c_int),
        "gs_default_settings": ([S], None),
        "gs_targets_layout": ([V, i32, T, i32, C.POINTER(C.c_int64), C.POINTER(C.c_int32)], C.c_int),
        "gs_workspace_query": ([S, i64, i32, T, i32, i64, C.POINTER(gs_sizes)], C.c_int),
        "gs_preprocess": ([S, vp, i64, i64, vp, i32, vp, vp], C.c_int),
        "gs_bin_sort": ([S, vp, i64, i64, i32, vp, i32, i32, vp, i64, vp, vp], C.c_int),
        "gs_render_fwd": ([S, vp, i64, i32, vp, i64, vp, i32, i32, vp, vp, vp, vp, vp, vp], C.c_int),
        "gs_render_bwd": ([S, vp, i64, i64, vp, i32, vp, vp, i64, vp, i32, i32, vp, vp, vp, vp,
                           vp, vp], C.c_int),
        "gs_raster_bwd": ([S, vp, i64, i32, vp, i64, vp, i32, i32, vp, vp, vp, vp, vp], C.c_int),
        "gs_render_fwd_store": ([S, vp, i64, i32, vp, i64, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp, i64, vp],
                                C.c_int),
        "gs_raster_bwd_stored": ([S, vp, i64, i32, vp, i64, vp, i32, i32, vp, vp, vp, vp, i64, vp, vp, vp],
                                 C.c_int),
        "gs_project_bwd": ([S, vp, i64, i64, vp, i32, vp, vp, vp], C.c_int),
        "gs_project_bwd_adam": ([S, vp, i64, i64, vp, i32, vp, vp, vp, C.POINTER(C.c_float), C.c_double,
                                 C.c_double, C.c_double, i32, vp, vp, vp], C.c_int),
        "gs_render_bwd_adam": ([S, vp, i64, i64, vp, i32, vp, vp, i64, vp, i32, i32, vp, vp, vp, vp,
                                vp, vp, C.POINTER(C.c_float), C.c_double, C.c_double, C.c_double,
                                i32, vp, vp, vp], C.c_int),
        "gs_pyramid_build": ([vp, i32, i32, i32, i32, vp, vp], C.c_int),
        "gs_pyramid_loss": ([vp, vp, vp, i32, i32, i64, f32, vp, vp, vp, vp, vp], C.c_int),
        "gs_adam_step": ([vp, vp, vp, vp, i64, i64, C.POINTER(C.c_float), C.c_double, C.c_double,
                          C.c_double, i32, vp, vp], C.c_int),
        "gs_step_advance": ([vp, vp], C.c_int),
        "gs_init_features": ([vp, i32, i32, vp, i32, vp, vp, vp], C.c_int),
        "gs_init_mlp_fwd": ([vp, vp, vp, i32, vp, vp, vp], C.c_int),
        "gs_init_mlp_bwd": ([vp, vp, vp, vp, i32, vp, vp, vp], C.c_int),
        "gs_init_mlp_adam": ([vp, vp, vp, vp, vp, vp, vp, f32, C.c_double, C.c_double, C.c_double, i32,
                              vp], C.c_int),
        "gs_to_bf16": ([vp, vp, i64, vp], C.c_int),
        "gs_init_heuristic": ([vp, vp, i32, vp, i64, i64, vp, vp], C.c_int),
        "gs_init_decode": ([vp, vp, V, i32, vp, vp, vp, vp], C.c_int),
        "gs_append": ([vp, vp, vp, i64, i64, vp, i32, vp], C.c_int),
        "gs_fill": ([vp, i64, f32, vp], C.c_int),
        "gs_densify_rule_make": ([C.c_double] * 6 + [C.POINTER(gs_densify_rule)], C.c_int),
        "gs_densify_stats": ([vp, i64, i64, vp, i32, vp, vp], C.c_int),
        "gs_densify_workspace_bytes": ([i64], C.c_size_t),
        "gs_densify": ([C.POINTER(gs_densify_rule), vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, i64, vp,
                        vp, vp], C.c_int),
        "gs_densify_noalloc": ([C.POINTER(gs_densify_rule), vp, vp, vp, vp, vp, i64, i64, vp, vp, vp, i64,
                                vp, vp], C.c_int),
        "gs_reset_opacity": ([vp, vp, vp, i64, i64, C.c_double, vp], C.c_int),
        "gs_sim3_workspace_bytes": ([i32], C.c_size_t),
        "gs_sim3_apply": ([vp, i64, i64, vp, i32, vp, vp, vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()
EXPORTED = ["gs_status_string", "gs_status_word", "gs_default_settings", "gs_targets_layout", "gs_workspace_query",
            "gs_preprocess", "gs_bin_sort", "gs_render_fwd", "gs_raster_bwd", "gs_render_fwd_store",
            "gs_raster_bwd_stored", "gs_project_bwd",
            "gs_project_bwd_adam", "gs_render_bwd", "gs_render_bwd_adam",
            "gs_pyramid_build",
            "gs_pyramid_loss", "gs_adam_step", "gs_step_advance", "gs_fill", "gs_init_features",
            "gs_init_mlp_fwd", "gs_init_mlp_bwd", "gs_init_mlp_adam", "gs_to_bf16", "gs_init_heuristic",
            "gs_init_decode", "gs_append", "gs_densify_rule_make", "gs_densify_stats",
            "gs_densify_workspace_bytes", "gs_densify", "gs_densify_noalloc", "gs_reset_opacity", "gs_sim3_workspace_bytes",
            "gs_sim3_apply"]


def _check(status: int, what: str):
    if status != 0:
        raise GsError(f"{what}: {_lib.gs_status_string(status).decode()} ({status})")


def _p(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise GsError("expected a device tensor")
    return C.c_void_p(t.data_ptr())


def _typed(t, dtype, what, ndim=None, rows=None):
    """Device pointer of a contiguous tensor of the given dtype (and shape)."""
    if t is None:
        return None
    if t.dtype != dtype:
        raise GsError(f"{what}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise GsError(f"{what}: expected a contiguous tensor")
    if ndim is not None and t.dim() != ndim:
        raise GsError(f"{what}: expected {ndim} dimensions, got {t.dim()}")
    if rows is not None and t.shape[0] != rows:
        raise GsError(f"{what}: expected {rows} rows, got {t.shape[0]}")
    return _p(t)


def _store(t, what, like=None):
    """A [59][n_cap] float32 parameter-layout tensor (params, grad, m, v)."""
    ptr = _typed(t, torch.float32, what, 2, NUM_ROWS)
    if like is not None and t is not None and t.shape != like.shape:
        raise GsError(f"{what}: shape {tuple(t.shape)} differs from the parameters' {tuple(like.shape)}")
    return ptr


def _f32(t, what):
    return _typed(t, torch.float32, what)


def _i32(t, what):
    return _typed(t, torch.int32, what)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def default_settings(**overrides) -> gs_settings:
    """Library defaults with overrides; ``status`` may be a device int32/uint32
    tensor of one element (checked mode's status word)."""
    s = gs_settings()
    _lib.gs_default_settings(C.byref(s))
    for k, v in overrides.items():
        if k == "status" and isinstance(v, torch.Tensor):
            v = _p(v).value
        setattr(s, k, v)
    return s


def gs_status_word(word: int) -> int:
    """Status code a device status word read back by the caller stands for."""
    return int(_lib.gs_status_word(C.c_uint32(int(word) & 0xffffffff)))


def check_status_word(word: int, what: str = "device status"):
    """Raises GsError when the status word reports an overflow or a non-finite value."""
    _check(gs_status_word(word), what)


def make_view(cam: dict) -> gs_view:
    v = gs_view()
    R = [float(x) for x in list(_flat(cam["R"]))]
    for i in range(9):
        v.R[i] = R[i]
    t = [float(x) for x in list(_flat(cam["t"]))]
    for i in range(3):
        v.t[i] = t[i]
    v.fx, v.fy, v.cx, v.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    v.width, v.height = int(cam["width"]), int(cam["height"])
    return v


def _flat(a):
    try:
        import numpy as np

        return np.asarray(a, dtype=np.float64).reshape(-1)
    except Exception:  # pragma: no cover
        return a


def gs_targets_layout(views, specs, tile_w: int = TILE):
    """specs: list of (view, level, bg(3), weight); tiles of tile_w x (256 / tile_w)
    pixels.  Returns (targets array, total_pixels, total_tiles)."""
    nv = len(views)
    varr = (gs_view * nv)(*views)
    tarr = (gs_target * len(specs))()
    for i, (view, level, bg, weight) in enumerate(specs):
        tarr[i].view, tarr[i].level, tarr[i].weight = int(view), int(level), float(weight)
        tarr[i].tile_w = int(tile_w)
        for c in range(3):
            tarr[i].bg[c] = float(bg[c])
    tp, tt = C.c_int64(), C.c_int32()
    _check(_lib.gs_targets_layout(varr, nv, tarr, len(specs), C.byref(tp), C.byref(tt)),
           "gs_targets_layout")
    return tarr, int(tp.value), int(tt.value)


def gs_workspace_query(settings, n_cap, n_views, targets, pair_cap) -> gs_sizes:
    out = gs_sizes()
    _check(_lib.gs_workspace_query(C.byref(settings), n_cap, n_views, targets, len(targets),
                                   pair_cap, C.byref(out)), "gs_workspace_query")
    return out


def to_device_struct_array(arr, device="cuda") -> torch.Tensor:
    """Copies a ctypes struct array into a device byte tensor."""
    raw = bytes(C.string_at(C.addressof(arr), C.sizeof(arr)))
    host = torch.frombuffer(bytearray(raw), dtype=torch.uint8)
    return host.to(device)


def gs_preprocess(settings, params, n, views_dev, n_views, proj_ws, stream=None):
    _check(_lib.gs_preprocess(C.byref(settings), _store(params, "params"), n, params.shape[1], _p(views_dev),
                              n_views, _p(proj_ws), _stream(stream)), "gs_preprocess")


def gs_bin_sort(settings, proj_ws, n, n_cap, n_views, targets_dev, n_targets, total_tiles, sort_ws,
                pair_cap, status_dev=None, stream=None):
    _check(_lib.gs_bin_sort(C.byref(settings), _p(proj_ws), n, n_cap, n_views, _p(targets_dev),
                            n_targets, total_tiles, _p(sort_ws), pair_cap, _p(status_dev),
                            _stream(stream)), "gs_bin_sort")


def gs_render_fwd(settings, proj_ws, n_cap, n_views, sort_ws, pair_cap, targets_dev, n_targets,
                  total_tiles, out_rgb, out_T, out_last, out_ncontrib=None, stream=None, out_nevals=None):
    _check(_lib.gs_render_fwd(C.byref(settings), _p(proj_ws), n_cap, n_views, _p(sort_ws), pair_cap,
                              _p(targets_dev), n_targets, total_tiles, _f32(out_rgb, "out_rgb"),
                              _f32(out_T, "out_T"), _i32(out_last, "out_last"),
                              _i32(out_ncontrib, "out_ncontrib"), _i32(out_nevals, "out_nevals"),
                              _stream(stream)), "gs_render_fwd")


def gs_render_bwd(settings, params, n, views_dev, n_views, proj_ws, sort_ws, pair_cap, targets_dev,
                  n_targets, total_tiles, out_T, out_last, dL_drgb, accum_ws, grad, stream=None):
    _check(_lib.gs_render_bwd(C.byref(settings), _store(params, "params"), n, params.shape[1], _p(views_dev),
                              n_views, _p(proj_ws), _p(sort_ws), pair_cap, _p(targets_dev),
                              n_targets, total_tiles, _f32(out_T, "out_T"), _i32(out_last, "out_last"),
                              _f32(dL_drgb, "dL_drgb"), _p(accum_ws), _store(grad, "grad", params),
                              _stream(stream)), "gs_render_bwd")


def gs_raster_bwd(settings, proj_ws, n_cap, n_views, sort_ws, pair_cap, targets_dev, n_targets,
                  total_tiles, out_T, out_last, dL_drgb, accum_ws, stream=None):
    _check(_lib.gs_raster_bwd(C.byref(settings), _p(proj_ws), n_cap, n_views, _p(sort_ws), pair_cap,
                              _p(targets_dev), n_targets, total_tiles, _f32(out_T, "out_T"),
                              _i32(out_last, "out_last"), _f32(dL_drgb, "dL_drgb"), _p(accum_ws),
                              _stream(stream)), "gs_raster_bwd")


def gs_render_fwd_store(settings, proj_ws, n_cap, n_views, sort_ws, pair_cap, targets_dev, n_targets,
                        total_tiles, out_rgb, out_T, out_last, out_ncontrib, tile_steps, store_base, store,
                        stream=None):
    if tile_steps.dtype != torch.int32 or tile_steps.numel() < total_tiles:
        raise GsError("tile_steps must be int32 with total_tiles entries")
    if store_base.dtype != torch.int64 or store_base.numel() < total_tiles + 1:
        raise GsError("store_base must be int64 with total_tiles + 1 entries")
    _check(_lib.gs_render_fwd_store(C.byref(settings), _p(proj_ws), n_cap, n_views, _p(sort_ws), pair_cap,
                                    _p(targets_dev), n_targets, total_tiles, _f32(out_rgb, "out_rgb"),
                                    _f32(out_T, "out_T"), _i32(out_last, "out_last"),
                                    _i32(out_ncontrib, "out_ncontrib"), _p(tile_steps), _p(store_base),
                                    _f32(store, "store"), store.numel(), _stream(stream)),
           "gs_render_fwd_store")


def gs_raster_bwd_stored(settings, proj_ws, n_cap, n_views, sort_ws, pair_cap, targets_dev, n_targets,
                         total_tiles, out_last, out_ncontrib, store_base, store, dL_drgb, accum_ws,
                         stream=None):
    if store_base.dtype != torch.int64 or store_base.numel() < total_tiles + 1:
        raise GsError("store_base must be int64 with total_tiles + 1 entries")
    _check(_lib.gs_raster_bwd_stored(C.byref(settings), _p(proj_ws), n_cap, n_views, _p(sort_ws), pair_cap,
                                     _p(targets_dev), n_targets, total_tiles, _i32(out_last, "out_last"),
                                     _i32(out_ncontrib, "out_ncontrib"), _p(store_base),
                                     _f32(store, "store"), store.numel(), _f32(dL_drgb, "dL_drgb"),
                                     _p(accum_ws), _stream(stream)), "gs_raster_bwd_stored")


def gs_project_bwd(settings, params, n, views_dev, n_views, accum_ws, grad, stream=None):
    _check(_lib.gs_project_bwd(C.byref(settings), _store(params, "params"), n, params.shape[1], _p(views_dev),
                               n_views, _p(accum_ws), _store(grad, "grad", params), _stream(stream)),
           "gs_project_bwd")


def _step_args(step):
    """An int step, or a device int32 tensor holding it (graph replay)."""
    if isinstance(step, torch.Tensor):
        return 0, _p(step)
    return int(step), None


def gs_project_bwd_adam(settings, params, n, views_dev, n_views, accum_ws, m, v, lr_rows, step,
                        beta1=0.9, beta2=0.999, eps=1e-15, proj_out=None, stream=None):
    lr = (C.c_float * NUM_ROWS)(*[float(x) for x in lr_rows])
    st, dst = _step_args(step)
    _check(_lib.gs_project_bwd_adam(C.byref(settings), _store(params, "params"), n, params.shape[1],
                                    _p(views_dev), n_views, _p(accum_ws), _store(m, "m", params),
                                    _store(v, "v", params), lr, beta1, beta2, eps, st, dst,
                                    _p(proj_out), _stream(stream)), "gs_project_bwd_adam")


def gs_render_bwd_adam(settings, params, n, views_dev, n_views, proj_ws, sort_ws, pair_cap,
                       targets_dev, n_targets, total_tiles, out_T, out_last, dL_drgb, accum_ws, m, v,
                       lr_rows, step, beta1=0.9, beta2=0.999, eps=1e-15, proj_out=None, stream=None):
    lr = (C.c_float * NUM_ROWS)(*[float(x) for x in lr_rows])
    st, dst = _step_args(step)
    _check(_lib.gs_render_bwd_adam(C.byref(settings), _store(params, "params"), n, params.shape[1],
                                   _p(views_dev), n_views, _p(proj_ws), _p(sort_ws), pair_cap,
                                   _p(targets_dev), n_targets, total_tiles, _f32(out_T, "out_T"),
                                   _i32(out_last, "out_last"), _f32(dL_drgb, "dL_drgb"), _p(accum_ws),
                                   _store(m, "m", params), _store(v, "v", params), lr, beta1, beta2,
                                   eps, st, dst,
                                   _p(proj_out), _stream(stream)), "gs_render_bwd_adam")


def gs_pyramid_build(img, levels, out, stream=None):
    Cc, H, W = img.shape
    _check(_lib.gs_pyramid_build(_typed(img, torch.float32, "img", 3), Cc, H, W, levels, _f32(out, "out"),
                                 _stream(stream)),
           "gs_pyramid_build")


def gs_pyramid_loss(render, target, targets_dev, n_targets, total_tiles, total_pixels, lam, loss_ws,
                    d_loss, d_total, dL_drender, stream=None):
    _check(_lib.gs_pyramid_loss(_f32(render, "render"), _f32(target, "target"), _p(targets_dev), n_targets,
                                total_tiles, total_pixels, lam, _p(loss_ws), _f32(d_loss, "d_loss"),
                                _f32(d_total, "d_total"), _f32(dL_drender, "dL_drender"),
                                _stream(stream)), "gs_pyramid_loss")


def gs_adam_step(params, grad, m, v, n, lr_rows, step, beta1=0.9, beta2=0.999, eps=1e-15,
                 stream=None):
    lr = (C.c_float * NUM_ROWS)(*[float(x) for x in lr_rows])
    st, dst = _step_args(step)
    _check(_lib.gs_adam_step(_store(params, "params"), _store(grad, "grad", params), _store(m, "m", params),
                             _store(v, "v", params), n, params.shape[1], lr, beta1,
                             beta2, eps, st, dst, _stream(stream)), "gs_adam_step")


def gs_step_advance(d_step, stream=None):
    _check(_lib.gs_step_advance(_p(d_step), _stream(stream)), "gs_step_advance")


def gs_fill(dst, value, stream=None):
    _check(_lib.gs_fill(_p(dst), dst.numel(), float(value), _stream(stream)), "gs_fill")


# ---- initialiser -----------------------------------------------------------
def gs_init_features(img, kp, x_bf16, heuristic=None, stream=None):
    _, H, W = img.shape
    _check(_lib.gs_init_features(_p(img), H, W, _p(kp), kp.shape[0], _p(heuristic), _p(x_bf16),
                                 _stream(stream)), "gs_init_features")


def gs_init_mlp_fwd(w_bf16, bias, x_bf16, y, act_ws, stream=None):
    _check(_lib.gs_init_mlp_fwd(_p(w_bf16), _p(bias), _p(x_bf16), x_bf16.shape[0], _p(y), _p(act_ws),
                                _stream(stream)), "gs_init_mlp_fwd")


def gs_init_mlp_bwd(w_bf16, x_bf16, act_ws, dy, dw, db, stream=None):
    _check(_lib.gs_init_mlp_bwd(_p(w_bf16), _p(x_bf16), _p(act_ws), _p(dy), dy.shape[0], _p(dw), _p(db),
                                _stream(stream)), "gs_init_mlp_bwd")


def gs_init_mlp_adam(w_master, b_master, w_bf16, dw, db, m, v, lr, step, beta1=0.9, beta2=0.999,
                     eps=1e-8, stream=None):
    _check(_lib.gs_init_mlp_adam(_p(w_master), _p(b_master), _p(w_bf16), _p(dw), _p(db), _p(m), _p(v),
                                 float(lr), beta1, beta2, eps, int(step), _stream(stream)),
           "gs_init_mlp_adam")


def gs_to_bf16(src, dst, stream=None):
    _check(_lib.gs_to_bf16(_p(src), _p(dst), src.numel(), _stream(stream)), "gs_to_bf16")


def gs_init_heuristic(new_mu, new_rgb, params, n, out, stream=None):
    _check(_lib.gs_init_heuristic(_p(new_mu), _p(new_rgb), new_mu.shape[1], _p(params), n,
                                  params.shape[1], _p(out), _stream(stream)), "gs_init_heuristic")


def gs_init_decode(y, kp, view, heuristic, out, used_fallback=None, stream=None):
    _check(_lib.gs_init_decode(_p(y), _p(kp), C.byref(view), y.shape[0], _p(heuristic), _p(out),
                               _p(used_fallback), _stream(stream)), "gs_init_decode")


def gs_append(params, m, v, n, new_params, stream=None):
    _check(_lib.gs_append(_p(params), _p(m), _p(v), n, params.shape[1], _p(new_params),
                          new_params.shape[1], _stream(stream)), "gs_append")


def densify_rule(extent, grad_threshold=2e-4, percent_dense=0.01, min_opacity=0.005, big_fraction=0.1,
                 shrink=1.6) -> gs_densify_rule:
    """Thresholds of the densification rule (big_fraction None: no size pruning)."""
    r = gs_densify_rule()
    _check(_lib.gs_densify_rule_make(float(extent), float(grad_threshold), float(percent_dense),
                                     float(min_opacity), 0.0 if big_fraction is None else float(big_fraction),
                                     float(shrink), C.byref(r)), "gs_densify_rule_make")
    return r


def gs_densify_stats(accum_ws, n, n_cap, views_dev, n_views, stats, stream=None):
    _check(_lib.gs_densify_stats(_p(accum_ws), n, n_cap, _p(views_dev), n_views,
                                 _typed(stats, torch.float32, "stats", 2, 2), _stream(stream)),
           "gs_densify_stats")


def gs_densify_workspace_bytes(n) -> int:
    return int(_lib.gs_densify_workspace_bytes(n))


def gs_densify(rule, params, m, v, stats, noise, n, out_params, out_m, out_v, ws, d_counts, stream=None):
    if stats.shape[1] != params.shape[1] or noise.shape[1] != params.shape[1]:
        raise GsError("stats and noise need the parameters' column capacity")
    _check(_lib.gs_densify(C.byref(rule), _store(params, "params"), _store(m, "m", params),
                           _store(v, "v", params), _typed(stats, torch.float32, "stats", 2, 2),
                           _typed(noise, torch.float32, "noise", 2, 6), n, params.shape[1],
                           _store(out_params, "out_params"), _store(out_m, "out_m", out_params),
                           _store(out_v, "out_v", out_params), out_params.shape[1], _p(ws),
                           _typed(d_counts, torch.int64, "d_counts"), _stream(stream)), "gs_densify")


DENSIFY_NOALLOC_MAX_N = 16777216


def gs_densify_noalloc(rule, params, m, v, stats, noise, n, out_params, out_m, out_v, d_counts, stream=None):
    if stats.shape[1] != params.shape[1] or noise.shape[1] != params.shape[1]:
        raise GsError("stats and noise need the parameters' column capacity")
    _check(_lib.gs_densify_noalloc(C.byref(rule), _store(params, "params"), _store(m, "m", params),
                                   _store(v, "v", params), _typed(stats, torch.float32, "stats", 2, 2),
                                   _typed(noise, torch.float32, "noise", 2, 6), n, params.shape[1],
                                   _store(out_params, "out_params"), _store(out_m, "out_m", out_params),
                                   _store(out_v, "out_v", out_params), out_params.shape[1],
                                   _typed(d_counts, torch.int64, "d_counts"), _stream(stream)),
           "gs_densify_noalloc")


def gs_reset_opacity(params, m, v, n, max_opacity=0.01, stream=None):
    _check(_lib.gs_reset_opacity(_store(params, "params"), _store(m, "m", params), _store(v, "v", params),
                                 n, params.shape[1], float(max_opacity), _stream(stream)),
           "gs_reset_opacity")


def sim3_table(sims, device="cuda") -> torch.Tensor:
    """Device array of gs_sim3 from ((w, x, y, z), t, s) triples."""
    arr = (gs_sim3 * len(sims))()
    for i, (q, t, s) in enumerate(sims):
        arr[i].q[:] = [float(x) for x in q]
        arr[i].t[:] = [float(x) for x in t]
        arr[i].s = float(s)
    return to_device_struct_array(arr, device)


def gs_sim3_workspace_bytes(n_transforms) -> int:
    return int(_lib.gs_sim3_workspace_bytes(n_transforms))


def gs_sim3_apply(params, n, transforms_dev, n_transforms, ws, assign=None, stream=None):
    if assign is not None and assign.numel() < n:
        raise GsError("assign needs one entry per primitive")
    if transforms_dev.numel() * transforms_dev.element_size() < n_transforms * C.sizeof(gs_sim3):
        raise GsError("transform array too small")
    if ws.numel() * ws.element_size() < gs_sim3_workspace_bytes(n_transforms):
        raise GsError("workspace too small")
    _check(_lib.gs_sim3_apply(_store(params, "params"), n, params.shape[1], _p(transforms_dev), n_transforms,
                              _i32(assign, "assign"), _p(ws), _stream(stream)), "gs_sim3_apply")
