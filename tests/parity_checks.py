"""GPU-vs-oracle comparisons whose tolerances come from counted discrete
differences: the registration quality block (Section III-C: inlier ratio,
rms of the inlier residuals, truncated cost) within the counted
correspondence mismatches, and the keyframe fusion (Section III-C) within the
keyframe pixels whose FP64 projection or gate value lies at a boundary."""
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


def _rays(g):
    el = g.el_top - np.arange(g.rows) * g.d_el
    az = 2 * np.pi * np.arange(g.cols) / g.cols
    E, A = np.meshgrid(el, az, indexing="ij")
    return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1)


def _proj(g, x):
    """Fractional pixel coordinates (fi, fj) of points x[..., 3] (FP64)."""
    el = np.arctan2(x[..., 2], np.hypot(x[..., 0], x[..., 1]))
    az = np.arctan2(x[..., 1], x[..., 0]) % (2 * np.pi)
    return (g.el_top - el) / g.d_el, az * g.cols / (2 * np.pi)


def _near_half(f, eps):
    return np.abs(f - np.floor(f) - 0.5) < eps


def _surfel_ok(g, s):
    return (s[..., 3] > g.r_min) & (s[..., 3] <= g.r_max) & (np.abs(s[..., :3]).sum(-1) > 0)


def fusion_ambiguous(sg, scan, kg, kf, cnt, T, fp=None, eps_px=1e-3, eps=1e-5):
    """Keyframe pixels whose fused value may differ between an FP32 and an
    FP64 implementation of the same fusion at pose T (scan -> keyframe):

    * update pass (pixels holding samples): the keyframe point taken into the
      scan projects within eps_px of a scan pixel boundary, or a gate (0.2 m
      distance, 30 deg normal, incidence) is within eps of its threshold;
    * fill pass (empty pixels): a scan point projects within eps_px of the
      pixel's boundary (the pixel and its 8 neighbours are marked), or the
      nearest two candidate ranges are within eps relative.

    FP32 rounding moves a projection by far less than 1e-3 pixel and a gate
    value by far less than 1e-5 at these ranges."""
    fp = fp or O.FuseParams()
    R, t = T[:3, :3], T[:3, 3]
    Uk, Us = _rays(kg), _rays(sg)
    H, W = sg.rows, sg.cols
    amb = np.zeros((kg.rows, kg.cols), bool)
    # update pass
    upd = (cnt > 0) & _surfel_ok(kg, kf)
    x1 = kf[..., 3:4] * Uk
    x = (x1 - t) @ R
    fi, fj = _proj(sg, x)
    near = _near_half(fi, eps_px) | _near_half(fj, eps_px)
    si = np.floor(fi + 0.5).astype(np.int64)
    sj = np.floor(fj + 0.5).astype(np.int64) % W
    inrow = (si >= 0) & (si < H)
    s2 = scan[np.clip(si, 0, H - 1), sj]
    ok2 = inrow & _surfel_ok(sg, s2)
    q = (s2[..., 3:4] * Us[np.clip(si, 0, H - 1), sj]) @ R.T + t
    m = s2[..., :3] @ R.T
    dist = np.linalg.norm(q - x1, axis=-1)
    cm = (m * kf[..., :3]).sum(-1)
    un = np.abs((Uk * kf[..., :3]).sum(-1))
    gate = (np.abs(dist - fp.d_max) < eps) | (np.abs(cm - fp.cos_theta_max) < eps) | (
        np.abs(un - fp.min_cos_incidence) < eps)
    amb |= upd & (near | (ok2 & gate))
    # fill pass
    empty = cnt == 0
    ok = _surfel_ok(sg, scan)
    qs = (scan[..., 3:4] * Us) @ R.T + t
    rq = np.linalg.norm(qs, axis=-1)
    ok &= (rq > kg.r_min) & (rq <= kg.r_max)
    gi, gj = _proj(kg, qs)
    ki = np.floor(gi + 0.5).astype(np.int64)
    kj = np.floor(gj + 0.5).astype(np.int64) % kg.cols
    ok_row = ok & (ki >= 0) & (ki < kg.rows)
    nearf = ok & (_near_half(gi, eps_px) | _near_half(gj, eps_px))
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            ii = np.clip(ki[nearf] + di, 0, kg.rows - 1)
            jj = (kj[nearf] + dj) % kg.cols
            amb[ii, jj] |= empty[ii, jj]
    kp = (ki * kg.cols + kj)[ok_row]
    rr = rq[ok_row]
    order = np.lexsort((rr, kp))
    kp, rr = kp[order], rr[order]
    same_next = kp[1:] == kp[:-1]
    first = np.r_[True, ~same_next]
    # the first two candidates of each pixel, in range order
    tie = same_next & first[:-1] & (np.abs(rr[1:] - rr[:-1]) <= eps * rr[:-1])
    hit = kp[:-1][tie]
    amb.reshape(-1)[hit] |= empty.reshape(-1)[hit]
    return amb


def assert_fusion_close(kg_gpu, cnt_gpu, kf_orc, cnt_orc, amb, dr_tol=1e-5, dn_tol=1e-4):
    """Fused keyframes (surfels and counts) of the GPU and the oracle: equal
    counts, ranges within dr_tol relative and normals within dn_tol, except
    at the ambiguous pixels of fusion_ambiguous."""
    diff = cnt_gpu != cnt_orc
    both = (cnt_orc > 0) & (cnt_gpu > 0)
    rel = np.zeros(cnt_orc.shape)
    rel[both] = np.abs(kg_gpu[..., 3][both] - kf_orc[..., 3][both]) / kf_orc[..., 3][both]
    dn = np.linalg.norm(kg_gpu[..., :3] - kf_orc[..., :3], axis=-1)
    diff |= both & ((rel > dr_tol) | (dn > dn_tol))
    unexplained = diff & ~amb
    return int(diff.sum()), int(amb.sum()), int(unexplained.sum())


def association_ambiguous(g, scan, kg, kf, T, d_max, cos_t, eps_px=1e-3, eps=1e-5, eps_dist=1e-4):
    """Scan pixels whose Omega-inlier decision at pose T (Section III-B) may
    differ between FP32 and FP64: the point projects within eps_px of a
    keyframe pixel boundary, the distance is within eps_dist (metres; FP32
    points at 50 m carry about 1e-5 m of rounding) or the normal gate value
    within eps of its threshold.  Returns the boolean mask (FP64, numpy
    only)."""
    R, t = T[:3, :3], T[:3, 3]
    ok = _surfel_ok(g, scan)
    q = (scan[..., 3:4] * _rays(g)) @ R.T + t
    m = scan[..., :3] @ R.T
    fi, fj = _proj(kg, q)
    near = _near_half(fi, eps_px) | _near_half(fj, eps_px)
    ki = np.floor(fi + 0.5).astype(np.int64)
    kj = np.floor(fj + 0.5).astype(np.int64) % kg.cols
    inrow = (ki >= 0) & (ki < kg.rows)
    kic = np.clip(ki, 0, kg.rows - 1)
    s1 = kf[kic, kj]
    x1 = s1[..., 3:4] * _rays(kg)[kic, kj]
    dist = np.linalg.norm(q - x1, axis=-1)
    cm = (m * s1[..., :3]).sum(-1)
    gate = inrow & _surfel_ok(kg, s1) & ((np.abs(dist - d_max) < eps_dist) | (np.abs(cm - cos_t) < eps))
    return ok & (near | gate)


def assert_scores_match(scores, ref, amb):
    """Integer candidate scores against the oracle's counts: each within its
    count of ambiguous pixels; the winner (the first maximum) is a candidate
    that the counts allow to be the maximum, and it is the oracle's own
    winner wherever the oracle's margin exceeds the ambiguity."""
    scores, ref, amb = np.asarray(scores), np.asarray(ref), np.asarray(amb)
    dev = np.abs(scores - ref)
    assert (dev <= amb).all(), (int(dev.max()), int(amb[np.argmax(dev - amb)]))
    c = int(np.argmax(scores))
    lo, hi = ref - amb, ref + amb
    assert hi[c] >= lo.max(), (c, hi[c], lo.max())
    c_ref = int(np.argmax(ref))
    others = np.delete(hi, c_ref)
    if others.size == 0 or lo[c_ref] > others.max():
        assert c == c_ref, (c, c_ref)
    return int(dev.sum()), int(amb.sum())
