"""Sweep intake (UPSLAM Section III-A): the per-column transforms that move
the measurements of one sweep into the frame of a single instant.

A sweep fires its columns one after the other (column j at the fraction
j / cols of the sweep period).  The paper corrects the orientation of every
measurement to a common instant from the gyroscope, on the CPU; these are
those host computations -- from gyroscope samples (rotation only) or from a
constant body twist (rotation and translation, e.g. the velocity of a motion
prior).  The projection into the panorama runs on the GPU
(``splat_sweep``).  Transforms map column j's frame into the reference frame.
"""
from __future__ import annotations

import numpy as np


def _hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def so3_exp(w) -> np.ndarray:
    """Rotation matrix of the rotation vector w (Rodrigues; Taylor series of
    the coefficients below 1e-4 rad)."""
    w = np.asarray(w, dtype=np.float64)
    th2 = float(w @ w)
    th = np.sqrt(th2)
    if th < 1e-4:
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0
    else:
        A = np.sin(th) / th
        B = (1.0 - np.cos(th)) / th2
    K = _hat(w)
    return np.eye(3) + A * K + B * (K @ K)


def se3_exp(xi) -> np.ndarray:
    """4x4 transform Exp of the twist xi = (omega, v)."""
    xi = np.asarray(xi, dtype=np.float64)
    w, v = xi[:3], xi[3:]
    th2 = float(w @ w)
    th = np.sqrt(th2)
    if th < 1e-4:
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0
    else:
        B = (1.0 - np.cos(th)) / th2
        C = (th - np.sin(th)) / (th2 * th)
    K = _hat(w)
    T = np.eye(4)
    T[:3, :3] = so3_exp(w)
    T[:3, 3] = (np.eye(3) + B * K + C * (K @ K)) @ v
    return T


def column_times(cols: int) -> np.ndarray:
    """Firing instants of the columns as fractions of the sweep period."""
    return np.arange(cols, dtype=np.float64) / cols


def twist_transforms(cols: int, xi, period: float = 0.1, t_ref: float = 1.0) -> np.ndarray:
    """[cols, 4, 4]: Exp((t_j - t_ref) period xi) for a sensor moving with the
    constant body twist xi = (omega rad/s, v m/s) during the sweep."""
    xi = np.asarray(xi, dtype=np.float64)
    return np.stack([se3_exp((t - t_ref) * period * xi) for t in column_times(cols)])


def gyro_transforms(cols: int, gyro_t, gyro_w, period: float = 0.1, t_ref: float = 1.0) -> np.ndarray:
    """[cols, 4, 4] rotations from gyroscope samples: body rates gyro_w[k]
    (rad/s) held from gyro_t[k] (s, sweep start = 0; increasing) to the next
    sample, the first one from the sweep start.  The
    orientation R(t) is integrated from the sweep start; column j's
    measurements move to the reference instant by R(t_ref)^T R(t_j)."""
    gt = np.asarray(gyro_t, dtype=np.float64)
    gw = np.asarray(gyro_w, dtype=np.float64).reshape(-1, 3)

    def orient(t):
        # sample k's rate holds from gyro_t[k] (the first one from 0) to the next sample
        R = np.eye(3)
        for k in range(len(gt)):
            a = 0.0 if k == 0 else gt[k]
            b = gt[k + 1] if k + 1 < len(gt) else np.inf
            if t <= a:
                break
            R = R @ so3_exp(gw[k] * (min(b, t) - a))
        return R

    R_ref = orient(t_ref * period)
    out = np.tile(np.eye(4), (cols, 1, 1))
    for j, t in enumerate(column_times(cols)):
        out[j, :3, :3] = R_ref.T @ orient(t * period)
    return out


def pack(col_T) -> np.ndarray:
    """float32 [cols, 12] (R row-major, t) as ``splat_sweep`` takes them."""
    a = np.asarray(col_T, dtype=np.float64)
    return np.ascontiguousarray(np.concatenate([a[:, :3, :3].reshape(-1, 9), a[:, :3, 3]], axis=1),
                                dtype=np.float32)
