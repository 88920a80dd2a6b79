"""FP64 CPU oracle of the photorealistic-mapping path (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never does, and this
package never imports the GPU library: the two meet only at the seeded inputs
of ``scenes``.

The arithmetic lives in ``gs_oracle.c`` (plain C, FP64, OpenMP over pixels),
compiled with gcc into ``_gs_oracle.so`` by :func:`build`.  This module only
marshals numpy arrays through ctypes.  Section/equation citations are in the C
source.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "_gs_oracle.so")
_lib = None

NROWS = 59
# record columns of preprocess()
REC_FIELDS = ["valid", "mx", "my", "z", "ca", "cb", "cc", "opacity", "r", "g", "b",
              "clamp_r", "clamp_g", "clamp_b", "s00", "s01", "s11", "extx", "exty", "cond"]
AMB_IMAGE, AMB_COUNT = 1, 2

DEFAULT_SETTINGS = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, t_min=1e-4, znear=0.2,
                        dilation=0.3, fov_clamp=1.3, sh_degree=3)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = C.CDLL(_LIB)
        dp, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int64)
        u8p, i32p = C.POINTER(C.c_uint8), C.POINTER(C.c_int32)
        lib.orc_preprocess.argtypes = [dp, C.c_int64, C.c_int64, dp, dp, dp]
        lib.orc_render.argtypes = [dp, C.c_int64, C.c_int64, dp, dp, C.c_int, u8p, dp, dp, i32p,
                                   u8p, i64p]
        lib.orc_pixel_list.argtypes = [dp, C.c_int64, C.c_int64, dp, dp, C.c_int, C.c_int, i64p,
                                       C.c_int]
        lib.orc_pixel_list.restype = C.c_int
        lib.orc_render_backward.argtypes = [dp, C.c_int64, C.c_int64, dp, dp, u8p, dp, dp, dp]
        lib.orc_gauss_backward.argtypes = [dp, C.c_int64, C.c_int64, dp, dp, dp, dp]
        lib.orc_pyr_down.argtypes = [dp, C.c_int, C.c_int, C.c_int, dp]
        lib.orc_loss.argtypes = [dp, dp, C.c_int, C.c_int, C.c_int, C.c_double, dp, dp]
        lib.orc_loss.restype = C.c_double
        lib.orc_adam.argtypes = [dp, dp, dp, dp, C.c_int64, C.c_int64, dp, C.c_double,
                                 C.c_double, C.c_double, C.c_int]
        lib.orc_sh_basis.argtypes = [C.c_int, dp, dp, dp]
        lib.orc_fd_gauss.argtypes = [dp, C.c_int64, C.c_int64, dp, dp, dp, i64p, C.c_int, i32p,
                                     C.c_int, C.c_double, dp, i32p]
        lib.orc_num_threads.restype = C.c_int
        lib.orc_set_threads.argtypes = [C.c_int]
        _lib = lib
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def cam_vec(cam: dict) -> np.ndarray:
    """Flatten a camera dict to the oracle's 23 doubles.

    Optional keys ``tan_half_fov_x``/``tan_half_fov_y`` set the field-of-view
    clamp explicitly (a pyramid level keeps its keyframe's level-0 values)."""
    v = np.zeros(23, np.float64)
    v[0:9] = np.asarray(cam["R"], np.float64).reshape(9)
    v[9:12] = np.asarray(cam["t"], np.float64)
    v[12:16] = [cam["fx"], cam["fy"], cam["cx"], cam["cy"]]
    v[16:18] = [cam["width"], cam["height"]]
    v[18:21] = np.asarray(cam.get("bg", (0, 0, 0)), np.float64)
    v[21] = cam.get("tan_half_fov_x", 0.0)
    v[22] = cam.get("tan_half_fov_y", 0.0)
    return v


def set_vec(settings: dict | None = None) -> np.ndarray:
    s = dict(DEFAULT_SETTINGS)
    s.update(settings or {})
    return np.array([s["alpha_min"], s["alpha_max"], s["t_min"], s["znear"], s["dilation"],
                     s["fov_clamp"], s["sh_degree"]], np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Sets the number of OpenMP threads of later calls."""
    _load().orc_set_threads(int(n))


def preprocess(params, n: int, cam: dict, settings=None) -> np.ndarray:
    """Per-Gaussian projection records, ``[n, len(REC_FIELDS)]`` float64."""
    lib = _load()
    P = _f64(params)
    rec = np.zeros((n, len(REC_FIELDS)), np.float64)
    lib.orc_preprocess(_ptr(P, C.c_double), n, P.shape[1], _ptr(cam_vec(cam), C.c_double),
                       _ptr(set_vec(settings), C.c_double), _ptr(rec, C.c_double))
    return rec


def render(params, n: int, cam: dict, settings=None, mask=None, prune: bool = True) -> dict:
    """Eq. 3 rendering.  Returns img [3,H,W], T [H,W], n_contrib [H,W], amb [H,W], counts."""
    lib = _load()
    P = _f64(params)
    H, W = cam["height"], cam["width"]
    img = np.zeros((3, H, W), np.float64)
    T = np.zeros((H, W), np.float64)
    nc = np.zeros((H, W), np.int32)
    amb = np.zeros((H, W), np.uint8)
    counts = np.zeros(5, np.int64)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    lib.orc_render(_ptr(P, C.c_double), n, P.shape[1], _ptr(cam_vec(cam), C.c_double),
                   _ptr(set_vec(settings), C.c_double), int(prune), _ptr(m, C.c_uint8),
                   _ptr(img, C.c_double), _ptr(T, C.c_double), _ptr(nc, C.c_int32),
                   _ptr(amb, C.c_uint8), _ptr(counts, C.c_int64))
    return dict(img=img, T=T, n_contrib=nc, amb=amb,
                counts=dict(evaluated=int(counts[0]), contributing=int(counts[1]),
                            composited=int(counts[2]), amb_image=int(counts[3]),
                            amb_count=int(counts[4])))


def pixel_list(params, n: int, cam: dict, px: int, py: int, settings=None, cap: int = 4096):
    """Ids of the Gaussians composited at pixel (px, py), front to back."""
    lib = _load()
    P = _f64(params)
    ids = np.zeros(cap, np.int64)
    k = lib.orc_pixel_list(_ptr(P, C.c_double), n, P.shape[1], _ptr(cam_vec(cam), C.c_double),
                           _ptr(set_vec(settings), C.c_double), px, py, _ptr(ids, C.c_int64), cap)
    return ids[:min(k, cap)]


def render_backward(params, n: int, cam: dict, dL_dimg, settings=None, mask=None,
                    with_2d: bool = False):
    """Gradient of <dL_dimg, render> w.r.t. the raw parameters, ``[59, n_cap]`` float64.

    With ``with_2d`` also returns the per-Gaussian 2D gradients ``[n, 9]``
    (d mean x, d mean y, d conic a, b, c, d opacity, d r, g, b).
    """
    lib = _load()
    P = _f64(params)
    g = np.zeros((NROWS, P.shape[1]), np.float64)
    g2 = np.zeros((max(n, 1), 9), np.float64) if with_2d else None
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    d = _f64(dL_dimg)
    lib.orc_render_backward(_ptr(P, C.c_double), n, P.shape[1], _ptr(cam_vec(cam), C.c_double),
                            _ptr(set_vec(settings), C.c_double), _ptr(m, C.c_uint8),
                            _ptr(d, C.c_double), _ptr(g, C.c_double), _ptr(g2, C.c_double))
    return (g, g2[:n]) if with_2d else g


def gauss_backward(params, g: int, cam: dict, g2, settings=None) -> np.ndarray:
    """Chain rule of Gaussian ``g`` from 2D gradients (9 values) to its 59 raw-parameter gradients."""
    lib = _load()
    P = _f64(params)
    out = np.zeros(NROWS, np.float64)
    lib.orc_gauss_backward(_ptr(P, C.c_double), P.shape[1], g, _ptr(cam_vec(cam), C.c_double),
                           _ptr(set_vec(settings), C.c_double), _ptr(_f64(g2), C.c_double),
                           _ptr(out, C.c_double))
    return out


def pyr_down(img) -> np.ndarray:
    """One Gaussian-pyramid level down: [C,H,W] -> [C,ceil(H/2),ceil(W/2)]."""
    lib = _load()
    x = _f64(img)
    Cc, H, W = x.shape
    out = np.zeros((Cc, (H + 1) // 2, (W + 1) // 2), np.float64)
    lib.orc_pyr_down(_ptr(x, C.c_double), Cc, H, W, _ptr(out, C.c_double))
    return out


def pyramid(img, levels: int):
    out = [_f64(img)]
    for _ in range(1, levels):
        out.append(pyr_down(out[-1]))
    return out


def loss(x, y, lam: float = 0.2, grad: bool = True):
    """Eq. 4 loss of one image pair ([C,H,W]).  Returns (L, dL/dx or None, (l1, ssim))."""
    lib = _load()
    a, b = _f64(x), _f64(y)
    Cc, H, W = a.shape
    d = np.zeros_like(a) if grad else None
    parts = np.zeros(2, np.float64)
    L = lib.orc_loss(_ptr(a, C.c_double), _ptr(b, C.c_double), Cc, H, W, lam,
                     _ptr(d, C.c_double), _ptr(parts, C.c_double))
    return float(L), d, (float(parts[0]), float(parts[1]))


def adam(p, g, m, v, n: int, lr_rows, step: int, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step on [59, n_cap] float64 arrays (copies returned)."""
    lib = _load()
    p, m, v = _f64(p).copy(), _f64(m).copy(), _f64(v).copy()
    gg = _f64(g)
    lr = _f64(np.broadcast_to(np.asarray(lr_rows, np.float64), (NROWS,)))
    lib.orc_adam(_ptr(p, C.c_double), _ptr(gg, C.c_double), _ptr(m, C.c_double),
                 _ptr(v, C.c_double), n, p.shape[1], _ptr(lr, C.c_double), beta1, beta2, eps, step)
    return p, m, v


def sh_basis(d, deg: int = 3):
    """Real SH values Y[16] and polynomial gradients dY[16,3] at unit direction d."""
    lib = _load()
    dd = _f64(d)
    Y = np.zeros(16, np.float64)
    dY = np.zeros((16, 3), np.float64)
    lib.orc_sh_basis(deg, _ptr(dd, C.c_double), _ptr(Y, C.c_double), _ptr(dY, C.c_double))
    return Y, dY


def fd_gauss(params, n: int, cam: dict, W, gid, rows, h: float = 1e-4, settings=None):
    """Central differences of <W, I> w.r.t. rows of Gaussian(s) gid, re-rendering only
    each perturbed Gaussian's footprint.  gid: int -> (fd [nrows], changed [nrows]);
    sequence -> arrays [len(gid), nrows]."""
    lib = _load()
    P = _f64(params)
    single = np.ndim(gid) == 0
    gids = np.ascontiguousarray(np.atleast_1d(gid), dtype=np.int64)
    rr = np.ascontiguousarray(rows, dtype=np.int32)
    fd = np.zeros((len(gids), len(rr)), np.float64)
    ch = np.zeros((len(gids), len(rr)), np.int32)
    Wd = _f64(W)
    lib.orc_fd_gauss(_ptr(P, C.c_double), n, P.shape[1], _ptr(cam_vec(cam), C.c_double),
                     _ptr(set_vec(settings), C.c_double), _ptr(Wd, C.c_double),
                     _ptr(gids, C.c_int64), len(gids), _ptr(rr, C.c_int32), len(rr), h,
                     _ptr(fd, C.c_double), _ptr(ch, C.c_int32))
    if single:
        return fd[0], ch[0].astype(bool)
    return fd, ch.astype(bool)
