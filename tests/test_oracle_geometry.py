"""Pins of the oracle's panorama geometry (rays and spherical projection,
Section III-A / III-B: sweeps are panoramic images and correspondences are
found by projecting points into them).

The projection is checked against a brute-force nearest-pixel search over all
pixels of small panoramas, and the pixel -> ray -> pixel round trip must be
the identity.  Neither check reuses the oracle's arithmetic.
"""
import math

import numpy as np
import pytest

import oracle as O
from synth import Geom, lidar_geom


def _test_rays(g):
    """Pixel rays written from the geometry definition with numpy."""
    el = g.el_top - np.arange(g.rows) * g.d_el
    az = 2 * np.pi * np.arange(g.cols) / g.cols
    E, A = np.meshgrid(el, az, indexing="ij")
    return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1), E, A


def _brute_force_pixel(g, q):
    """Nearest row by elevation and nearest column by circular azimuth
    distance, searching every row and column."""
    el = math.atan2(q[2], math.hypot(q[0], q[1]))
    az = math.atan2(q[1], q[0]) % (2 * math.pi)
    rows_el = g.el_top - np.arange(g.rows) * g.d_el
    cols_az = 2 * np.pi * np.arange(g.cols) / g.cols
    di = np.abs(rows_el - el)
    da = np.abs((cols_az - az + np.pi) % (2 * np.pi) - np.pi)
    i = int(np.argmin(di))
    j = int(np.argmin(da))
    # out of the panorama when farther than half a row beyond the first/last row
    if el > g.el_top + g.d_el / 2 or el < g.el_top - (g.rows - 1) * g.d_el - g.d_el / 2:
        return None
    return i, j


def test_ray_matches_definition():
    g = lidar_geom(64, 512)
    U, _, _ = _test_rays(g)
    for i, j in [(0, 0), (5, 17), (63, 511), (31, 256)]:
        np.testing.assert_allclose(O.ray(g, i, j), U[i, j], atol=1e-15)


@pytest.mark.parametrize("rows,cols", [(8, 32), (64, 512), (128, 1024)])
def test_round_trip_identity(rows, cols):
    g = lidar_geom(rows, cols)
    U, _, _ = _test_rays(g)
    rng = np.random.default_rng(3)
    r = rng.uniform(0.6, 49.0, size=(rows, cols, 1))
    i, j, ok = O.project(g, (U * r).reshape(-1, 3))
    assert ok.all()
    I, J = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    assert np.array_equal(i.reshape(rows, cols), I)
    assert np.array_equal(j.reshape(rows, cols), J)


def test_projection_brute_force_8x32():
    g = Geom(8, 32, math.radians(10.0), math.radians(20.0) / 7, 0.0, 50.0)
    rng = np.random.default_rng(7)
    q = rng.normal(size=(4000, 3))
    q[:, 2] *= 0.25
    q *= rng.uniform(0.5, 40, size=(4000, 1))
    i, j, ok = O.project(g, q)
    n_in = 0
    for k in range(len(q)):
        bf = _brute_force_pixel(g, q[k])
        if bf is None:
            assert not ok[k]
        else:
            n_in += 1
            assert ok[k] and (i[k], j[k]) == bf, (k, q[k], (i[k], j[k]), bf)
    assert n_in > 1000


def test_projection_azimuth_wrap_and_origin():
    g = Geom(8, 32, math.radians(10.0), math.radians(20.0) / 7, 0.0, 50.0)
    # azimuth just below 2*pi rounds to column 0 (j = cols wraps)
    a = 2 * math.pi - 1e-4
    i, j, ok = O.project(g, [[math.cos(a), math.sin(a), 0.0]])
    assert ok[0] and j[0] == 0
    # the origin has no pixel
    _, _, ok = O.project(g, [[0.0, 0.0, 0.0]])
    assert not ok[0]
    # straight up is outside a +-10 degree panorama
    _, _, ok = O.project(g, [[0.0, 0.0, 1.0]])
    assert not ok[0]


def test_pyramid_level_keeps_angles():
    """Level-l pixel (i, j) is level-0 pixel (2^l i, 2^l j) and its ray under the
    level-l geometry is the same ray."""
    g = lidar_geom(64, 512)
    rng = np.random.default_rng(1)
    s = rng.normal(size=(64, 512, 4))
    for l in (1, 2):
        p = O.pyramid_level(g, s, l)
        assert np.array_equal(p, s[:: 1 << l, :: 1 << l])
        gl = g.level(l)
        for (i, j) in [(0, 0), (3, 7), (gl.rows - 1, gl.cols - 1)]:
            np.testing.assert_allclose(O.ray(gl, i, j), O.ray(g, i << l, j << l), atol=1e-15)
