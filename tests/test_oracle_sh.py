"""Pins of the oracle's spherical-harmonic colour (the colour "converted from SH", Eq. 3).

Orthonormality on the sphere by exact quadrature (Gauss-Legendre in cos(theta)
x uniform phi, exact for polynomials of degree <= 7), the DC-only closed form,
and the basis gradient against central differences.
"""

import numpy as np

import scenes


def _quadrature():
    xs, ws = np.polynomial.legendre.leggauss(8)
    nphi = 16
    phis = 2 * np.pi * np.arange(nphi) / nphi
    pts, wts = [], []
    for ct, w in zip(xs, ws):
        st = np.sqrt(1 - ct * ct)
        for ph in phis:
            pts.append([st * np.cos(ph), st * np.sin(ph), ct])
            wts.append(w * 2 * np.pi / nphi)
    return np.array(pts), np.array(wts)


def test_sh_orthonormal(orc):
    pts, wts = _quadrature()
    Y = np.array([orc.sh_basis(d)[0] for d in pts])      # [npts, 16]
    gram = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-13)


def test_sh_degree_truncation(orc):
    d = np.array([0.36, -0.48, 0.8])
    for deg, nk in [(0, 1), (1, 4), (2, 9), (3, 16)]:
        Y, _ = orc.sh_basis(d, deg)
        assert np.all(Y[nk:] == 0) and np.all(Y[:nk] != 0)


def test_sh_gradient_fd(orc):
    rng = np.random.default_rng(2)
    h = 1e-6
    for _ in range(10):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        _, dY = orc.sh_basis(d)
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            fd = (orc.sh_basis(d + e)[0] - orc.sh_basis(d - e)[0]) / (2 * h)
            np.testing.assert_allclose(dY[:, i], fd, atol=1e-8)


def test_dc_only_colour_is_view_independent(orc):
    """With only the DC coefficient, colour = 0.5 + dc / (2 sqrt(pi)) from every view."""
    n = 8
    p = np.zeros((59, 256))
    rng = np.random.default_rng(4)
    p[0:3, :n] = rng.uniform(-1, 1, (3, n)) + np.array([[0], [0], [5]])
    p[3:6, :n] = -3
    p[6, :n] = 1
    dc = rng.uniform(-0.5, 1.5, (3, n))
    p[11:14, :n] = dc
    expect = np.maximum(0.5 + dc / (2 * np.sqrt(np.pi)), 0)
    for ang in [0.0, 0.4, -0.3]:
        c, s = np.cos(ang), np.sin(ang)
        R = np.array([[c, 0, -s], [0, 1, 0], [s, 0, c]])
        cam = scenes.pinhole(64, 64, 64.0, R=R, t=[0.3, -0.2, 0.5])
        rec = orc.preprocess(p, n, cam)
        v = rec[:, 0] > 0
        assert v.any()
        np.testing.assert_allclose(rec[v, 8:11], expect.T[v], rtol=1e-14)
        np.testing.assert_array_equal(rec[v, 11:14], (0.5 + dc / (2 * np.sqrt(np.pi)) < 0).T[v])
