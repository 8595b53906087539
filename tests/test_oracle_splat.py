"""Pins of the oracle's panorama formation (Section III-A: the measurements
of a sweep are moved into the frame of one instant and projected into a
panoramic image, the nearest return per pixel).

* identity transforms into the same geometry give back the sweep;
* a yaw by exactly k columns rolls the image by k columns;
* brute force on 8 x 32: each measurement transformed with numpy, its pixel
  found by independent arg-mins over the row elevations and the column
  azimuths, the nearest (then the first) kept per pixel;
* de-skew: a sweep rendered from a turning sensor (90 deg/s over 0.1 s),
  moved with the true per-column transforms, matches the panorama rendered at
  the reference instant (94 % of the pixels within 2 cm), while the raw sweep
  and the sweep moved the wrong way do not.
"""
import math

import numpy as np
import pytest

import oracle as O
from synth import lidar_geom, rot_x, rot_z, se3
from synth import workloads as W


def test_identity_gives_back_the_sweep():
    c = W.config0()
    g = c["geom"]
    raw = c["scan"].astype(np.float64)
    out = O.splat_sweep(g, raw, None, g)
    v = raw > 0
    assert np.array_equal(out > 0, v)
    np.testing.assert_allclose(out[v], raw[v], rtol=1e-13)


def test_yaw_by_whole_columns_rolls():
    c = W.config0()
    g = c["geom"]
    raw = c["scan"].astype(np.float64)
    k = 7
    C = np.repeat(se3(rot_z(2 * math.pi * k / g.cols))[None], g.cols, 0)
    out = O.splat_sweep(g, raw, C, g)
    want = np.roll(raw, k, axis=1)
    assert np.array_equal(out > 0, want > 0)
    np.testing.assert_allclose(out[want > 0], want[want > 0], rtol=1e-12)


def test_brute_force_8x32():
    g = lidar_geom(8, 32)
    rng = np.random.default_rng(5)
    raw = rng.uniform(0.5, 20.0, size=(8, 32))
    raw[rng.random((8, 32)) < 0.1] = 0.0
    C = np.stack([se3(rot_z(rng.normal(0, 0.3)) @ rot_x(rng.normal(0, 0.05)), rng.normal(0, 0.3, 3))
                  for _ in range(32)])
    out = O.splat_sweep(g, raw, C, g)
    els = g.el_top - np.arange(g.rows) * g.d_el
    azs = 2 * np.pi * np.arange(g.cols) / g.cols
    best = {}
    for i in range(8):
        for j in range(32):
            r = raw[i, j]
            if not (0.0 < r <= g.r_max):
                continue
            el, az = els[i], azs[j]
            x = r * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
            y = C[j, :3, :3] @ x + C[j, :3, 3]
            ry = float(np.linalg.norm(y))
            if not (0.0 < ry <= g.r_max):
                continue
            e = math.atan2(y[2], math.hypot(y[0], y[1]))
            a = math.atan2(y[1], y[0]) % (2 * math.pi)
            if e > g.el_top + g.d_el / 2 or e < els[-1] - g.d_el / 2:
                continue
            oi = int(np.argmin(np.abs(els - e)))
            da = np.abs((azs - a + np.pi) % (2 * np.pi) - np.pi)
            oj = int(np.argmin(da))
            key = (oi, oj)
            cand = (ry, i * 32 + j)
            if key not in best or cand < best[key]:
                best[key] = cand
    want = np.zeros((8, 32))
    for (oi, oj), (ry, _) in best.items():
        want[oi, oj] = ry
    assert np.array_equal(out > 0, want > 0)
    np.testing.assert_allclose(out, want, rtol=1e-13)


@pytest.mark.parametrize("outdoor", [False, True])
def test_deskew_of_a_turning_sensor(outdoor):
    c = W.moving_sweep(outdoor=outdoor)
    g = c["geom"]
    ref = c["ref"].astype(np.float64)

    def close(img):
        both = (ref > 0) & (img > 0)
        return (np.abs(img - ref)[both] < 0.02).mean()

    good = close(O.splat_sweep(g, c["raw"], c["col_T"], g))
    raw = close(c["raw"].astype(np.float64))
    wrong = close(O.splat_sweep(g, c["raw"], np.linalg.inv(c["col_T"]), g))
    print(f"within 2 cm: de-skewed {good:.3f}, raw {raw:.3f}, wrong way {wrong:.3f}")
    assert good > 0.8 and raw < 0.6 and wrong < 0.6
