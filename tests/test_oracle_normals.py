"""Pins of the oracle's normal estimation (Section III-A: cross product of the
vectors to two image neighbours, then edge-aware a-trous smoothing).

* Any three points of a plane give the plane's normal: on rendered analytic
  planes the raw normal equals the plane normal (facing the sensor) to 1e-12.
* A-trous invariants: constant-normal regions are fixed points, outputs are
  unit length, invalid stays invalid, zero levels is the identity.
* In the limit of infinite edge-stopping widths the a-trous level is the
  normalised dilated B3-spline convolution, checked against scipy.
The exact edge-stopping weights themselves have no independent pin.
"""
import math

import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from synth import Geom, lidar_geom


def _rays(g):
    el = g.el_top - np.arange(g.rows) * g.d_el
    az = 2 * np.pi * np.arange(g.cols) / g.cols
    E, A = np.meshgrid(el, az, indexing="ij")
    return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1)


def _plane_depth(g, n, d):
    """Range image of the plane {x : n.x = d} seen from the origin."""
    U = _rays(g)
    den = U @ n
    with np.errstate(divide="ignore", invalid="ignore"):
        r = d / den
    r[(den == 0) | (r <= 0) | (r > g.r_max)] = 0.0
    return r


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_plane_normals_exact(seed):
    g = lidar_geom(64, 512, r_max=200.0)
    rng = np.random.default_rng(seed)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    d = rng.uniform(1.0, 5.0)
    depth = _plane_depth(g, n, d)
    s = O.raw_normals(g, depth, max_rel_jump=1e9)
    has = np.abs(s[..., :3]).sum(-1) > 0
    assert has.sum() > 1000
    # facing the sensor: the plane is at n.x = d > 0, so the sensor-facing normal is -n
    err = np.abs(s[has][:, :3] - (-n)).max()
    assert err < 1e-12, err
    # a-trous leaves a constant-normal image unchanged
    a = O.atrous(g, s, levels=2)
    np.testing.assert_allclose(a[has][:, :3], s[has][:, :3], atol=1e-13)
    assert np.array_equal(a[..., 3], s[..., 3])


def test_invalid_neighbours_and_jumps():
    g = lidar_geom(8, 32)
    depth = np.full((8, 32), 10.0)
    depth[3, 5] = 0.0                      # no return
    depth[6, 20] = 25.0                    # a 150 % range jump
    s = O.raw_normals(g, depth, max_rel_jump=0.5)
    has = np.abs(s[..., :3]).sum(-1) > 0
    # the invalid pixel and the pixels that use it as right / lower neighbour
    assert not has[3, 5] and not has[3, 4] and not has[2, 5]
    assert s[3, 5, 3] == 0.0
    # the jump cuts the pixels that use it as a neighbour (|25 - 10| > 0.5 * 10)
    # and the pixel itself (|10 - 25| > 0.5 * 25)
    assert not has[6, 19] and not has[5, 20] and not has[6, 20]
    # the test is relative to the centre range and inclusive: 10 m neighbours
    # of a 20 m pixel (a 50 % jump) are accepted
    d2 = np.full((8, 32), 10.0)
    d2[6, 20] = 20.0
    assert np.abs(O.raw_normals(g, d2, max_rel_jump=0.5)[6, 20, :3]).sum() > 0
    # everything else on the sphere of radius 10 has a normal pointing inward
    p = _rays(g) * depth[..., None]
    ok = has.copy()
    assert ok.sum() > 200
    assert (np.einsum("ijk,ijk->ij", s[..., :3], p)[ok] < 0).all()


def test_last_row_uses_previous_row():
    g = lidar_geom(8, 32, r_max=200.0)
    n = np.array([0.0, 0.0, 1.0])
    depth = _plane_depth(g, -n, 2.0)       # floor 2 m below
    s = O.raw_normals(g, depth, max_rel_jump=1e9)
    has = np.abs(s[..., :3]).sum(-1) > 0
    assert has[-1].all()
    np.testing.assert_allclose(s[-1, :, :3], np.tile(n, (32, 1)), atol=1e-12)


def _unit_random_surfels(g, seed, frac_invalid=0.1):
    rng = np.random.default_rng(seed)
    s = np.zeros((g.rows, g.cols, 4))
    v = rng.normal(size=(g.rows, g.cols, 3)) * 0.3 + np.array([0.0, 0.0, 1.0])
    v /= np.linalg.norm(v, axis=-1, keepdims=True)
    s[..., :3] = v
    s[..., 3] = rng.uniform(2.0, 20.0, size=(g.rows, g.cols))
    bad = rng.random((g.rows, g.cols)) < frac_invalid
    s[bad, :3] = 0.0
    return s, bad


def test_atrous_invariants():
    g = lidar_geom(32, 64)
    s, bad = _unit_random_surfels(g, 5)
    out = O.atrous(g, s, levels=2)
    has = np.abs(out[..., :3]).sum(-1) > 0
    assert np.array_equal(has, ~bad)
    np.testing.assert_allclose(np.linalg.norm(out[has][:, :3], axis=-1), 1.0, atol=1e-14)
    assert np.array_equal(out[..., 3], s[..., 3])
    assert np.array_equal(O.atrous(g, s, levels=0), s)


def _b3_dilated_kernel(step):
    h = np.array([1, 4, 6, 4, 1]) / 16.0
    k = np.zeros((4 * step + 1, 4 * step + 1))
    k[::step, ::step] = np.outer(h, h)
    return k


def _reference_smooth(s, step):
    """Normalised convolution with the dilated B3 kernel: rows outside the
    image contribute nothing (zero padding), columns wrap."""
    k = _b3_dilated_kernel(step)
    valid = (np.abs(s[..., :3]).sum(-1) > 0).astype(float)
    pad = 2 * step
    out = np.zeros_like(s)
    acc = []
    for c in range(3):
        x = np.pad(s[..., c] * valid, ((pad, pad), (0, 0)), mode="constant")
        x = np.pad(x, ((0, 0), (pad, pad)), mode="wrap")
        acc.append(ndimage.correlate(x, k, mode="constant")[pad:-pad, pad:-pad])
    acc = np.stack(acc, -1)
    nn = np.linalg.norm(acc, axis=-1, keepdims=True)
    out[..., :3] = np.where(valid[..., None] > 0, acc / np.where(nn > 0, nn, 1), 0.0)
    out[..., 3] = s[..., 3]
    return out


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_atrous_wide_weights_is_b3_convolution(levels):
    g = lidar_geom(32, 64)
    s, _ = _unit_random_surfels(g, 9)
    out = O.atrous(g, s, levels=levels, sigma_r=1e9, sigma_n=1e9)
    ref = s
    for l in range(levels):
        ref = _reference_smooth(ref, 1 << l)
    np.testing.assert_allclose(out, ref, atol=1e-12)


def test_edge_stopping_separates_two_planes():
    """Across a crease between two planes the normal weight exp(-(2-2cos)/sigma_n^2)
    is tiny: smoothing barely mixes the two normals (a property, not a value)."""
    g = lidar_geom(16, 64)
    s = np.zeros((16, 64, 4))
    s[..., 3] = 5.0
    s[:, :32, :3] = [0.0, 0.0, 1.0]
    s[:, 32:, :3] = [1.0, 0.0, 0.0]
    out = O.atrous(g, s, levels=2)
    left = out[:, 4:28, :3]
    assert np.abs(left - [0.0, 0.0, 1.0]).max() < 1e-3
    plain = O.atrous(g, s, levels=2, sigma_r=1e9, sigma_n=1e9)
    assert np.abs(plain[:, 30, :3] - [0.0, 0.0, 1.0]).max() > 0.1
