"""Comparison of the registration quality block (Section III-C: inlier ratio,
rms of the inlier residuals, truncated cost) between the GPU and the oracle,
with tolerances derived from the counted correspondence mismatches."""
import math

import numpy as np

import oracle as O
import synth


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _np(t):
    return t.detach().cpu().numpy()


def quality_mismatches(gpu_lib, ctx, g, scan, kf, T_gpu, T_orc, d_max=0.5):
    """Pixels whose (keyframe index, inlier) differ between the GPU's
    association at T_gpu and the oracle's at T_orc (level 0, the quality
    pass's thresholds)."""
    idx, inl = gpu_lib.correspondences(ctx, g, _t(scan), g, _t(kf), T_gpu, d_max=d_max)
    oi, oin = O.correspondences(g, scan, g, kf, T_orc, d_max)
    return int(((_np(idx) != oi) | (_np(inl).astype(bool) != oin)).sum())


def assert_quality_close(res, ref, mism, tau, dr=0.0, sum_abs_r=0.0):
    """The quality block (Section III-C) against the oracle's.  Each pixel
    whose correspondence differs moves the truncated cost and the inlier sum
    of r^2 by at most tau^2 (an inlier's |r| is at most d_max = tau) and the
    inlier count by one; a pose difference moving every point by at most dr
    changes an inlier's r^2 by at most 2|r| dr + dr^2; FP32 residuals add a
    relative 1e-5."""
    assert res["valid"] == ref["valid"]
    assert abs(res["inliers"] - ref["inliers"]) <= mism, (res["inliers"], ref["inliers"], mism)
    pose_term = 2.0 * sum_abs_r * dr + ref["inliers"] * dr * dr
    tol_e = mism * tau * tau + pose_term + 1e-5 * ref["trunc_cost"]
    assert abs(res["trunc_cost"] - ref["trunc_cost"]) <= tol_e, (res["trunc_cost"], ref["trunc_cost"], tol_e)
    s_gpu, s_orc = res["rms"] ** 2 * res["inliers"], ref["rms"] ** 2 * ref["inliers"]
    tol_s = mism * tau * tau + pose_term + 1e-5 * s_orc
    assert abs(s_gpu - s_orc) <= tol_s, (s_gpu, s_orc, tol_s)
    if ref["valid"]:
        assert abs(res["inlier_ratio"] - ref["inlier_ratio"]) <= mism / ref["valid"] + 1e-15


def pose_displacement_bound(T_a, T_b, max_range):
    """An upper bound on |T_a x - T_b x| for |x| <= max_range."""
    rot, tr = synth.pose_error(T_a, T_b)
    return tr + max_range * 2.0 * math.sin(rot / 2.0) + 1e-12
