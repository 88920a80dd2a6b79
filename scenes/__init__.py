"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws random numbers and builds camera poses; it holds none of the
rendering, loss or optimiser arithmetic.  Every array it returns is float32 (or
int32), laid out the way the library consumes it:

* ``params``: ``[59, n_cap]`` float32, structure-of-arrays.  Rows 0-2 mean
  (x, y, z), rows 3-5 log-scale, rows 6-9 quaternion (w, x, y, z), row 10 the
  opacity logit, rows ``11 + 3*k + ch`` spherical-harmonic coefficient ``k``
  (``0 <= k < 16``) of colour channel ``ch`` (R, G, B).  Columns ``>= n`` are
  padding and are zero.
* cameras: ``dict`` with ``R`` (3x3 world-to-camera, row-major), ``t`` (3),
  ``fx, fy, cx, cy`` (pixels; pixel ``(i, j)`` has its centre at ``(i, j)``),
  ``width``, ``height``, ``bg`` (3).

The distributions follow the workloads the paper's mapper faces (a room-sized
indoor map seen from keyframes at the Replica resolution 1200x680, Section 4.1),
with the per-parameter laws of the synthetic scene recipe described in the
design notes.  Draw order is fixed: means, log-scales, quaternions, opacity
logits, SH-DC, SH-rest, perturbations, poses.
"""

from .gen import (  # noqa: F401
    NROWS,
    ROW_MU,
    ROW_LOGS,
    ROW_QUAT,
    ROW_OPAC,
    ROW_SH,
    pad_cap,
    draw_gaussians,
    perturb,
    tiny_scene,
    room_scene,
    pinhole,
    random_walk,
    level_camera,
    smooth_image,
    mixed_keyframes,
    ROOM_LO,
    ROOM_HI,
    densify_case,
    degenerate_scene,
    DEGENERATE_KINDS,
)
