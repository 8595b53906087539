"""GPU-vs-oracle parity of the HIP path, called through the C ABI.

Floating point: the GPU computes per pixel in FP32, the oracle in FP64, so
per-pixel quantities agree to FP32 rounding (normals ~1e-5, ranges ~1e-6
relative).  Discrete decisions (pixel indices, Omega, validity) can flip where
the FP32 and FP64 values straddle a boundary: they must be bit-exact at the
identity pose, and elsewhere the number of flips is counted and bounded.
Poses must agree with the oracle to 1e-5 rad / 1e-5 m.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from synth import lidar_geom, se3, rot_z, rot_x
from synth import workloads as W
from parity_checks import assert_quality_close, pose_displacement_bound, quality_mismatches

pytestmark = pytest.mark.gpu

ROT_TOL = 1e-5
TR_TOL = 1e-5


def _t(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def torch_mod(gpu_lib):
    import torch
    return torch


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context(0, max_pixels=128 * 2048)
    yield c
    c.close()


@pytest.fixture(scope="module")
def c0():
    return W.config0()


@pytest.fixture(scope="module")
def c0_surfels(c0):
    """Oracle surfels of the config-0 pair, rounded to FP32: identical inputs
    for both registration implementations."""
    g = c0["geom"]
    kf = O.panorama_normals(g, c0["kf"]).astype(np.float32)
    scan = O.panorama_normals(g, c0["scan"]).astype(np.float32)
    return kf, scan


def _normal_mask(s):
    return np.abs(s[..., :3]).sum(-1) > 0


# ------------------------------------------------------------------ normals

@pytest.mark.parametrize("levels", [0, 1, 2])
def test_normals_parity(gpu_lib, ctx, c0, levels, torch_mod):
    g = c0["geom"]
    depth = c0["scan"]
    gs = _np(gpu_lib.panorama_normals(ctx, g, _t(depth), params=gpu_lib.NormalParams(atrous_levels=levels)))
    os_ = O.panorama_normals(g, depth, O.NormalParams(atrous_levels=levels))
    # ranges are copied: bit-exact
    assert np.array_equal(gs[..., 3], os_[..., 3].astype(np.float32))
    mg, mo = _normal_mask(gs), _normal_mask(os_)
    flips = int((mg != mo).sum())
    assert flips <= 5, flips
    both = mg & mo
    err = np.linalg.norm(gs[both][:, :3] - os_[both][:, :3], axis=-1)
    assert err.max() < 2e-4 and np.median(err) < 1e-5, (err.max(), np.median(err))


def test_normals_exact_plane(gpu_lib, ctx):
    g = lidar_geom(64, 512, r_max=200.0)
    el = g.el_top - np.arange(g.rows) * g.d_el
    az = 2 * np.pi * np.arange(g.cols) / g.cols
    E, A = np.meshgrid(el, az, indexing="ij")
    U = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1)
    n = np.array([0.3, -0.5, 0.8])
    n /= np.linalg.norm(n)
    den = U @ n
    r = np.where(den > 0.1, 3.0 / np.where(den > 0, den, 1), 0.0)
    r[r > g.r_max] = 0
    s = _np(gpu_lib.panorama_normals(ctx, g, _t(r.astype(np.float32)),
                                     params=gpu_lib.NormalParams(atrous_levels=2, max_rel_jump=1e9)))
    m = _normal_mask(s)
    assert m.sum() > 5000
    err = np.linalg.norm(s[m][:, :3] + n, axis=-1)
    print(f"exact plane: normal error max {err.max():.2e}, median {np.median(err):.2e} over {m.sum()} pixels")
    assert err.max() < 1e-5


def test_normals_invalid_inputs(gpu_lib, ctx, c0):
    """NaN, +-Inf, negative and out-of-range depths are no-returns."""
    g = c0["geom"]
    d = c0["scan"].copy()
    bad = [(3, 7, np.nan), (10, 100, np.inf), (20, 200, -np.inf), (30, 300, -2.0), (40, 400, 75.0)]
    for i, j, v in bad:
        d[i, j] = v
    s = _np(gpu_lib.panorama_normals(ctx, g, _t(d)))
    for i, j, _ in bad:
        assert s[i, j, 3] == 0.0 and not _normal_mask(s)[i, j]
    assert np.isfinite(s).all()


# ------------------------------------------------------------------ pyramid

def test_pyramid_bit_exact(gpu_lib, ctx, c0_surfels):
    kf, _ = c0_surfels
    g = lidar_geom(64, 512)
    for l in (1, 2, 3):
        out = _np(gpu_lib.pyramid_level(ctx, g, _t(kf), l))
        assert np.array_equal(out, O.pyramid_level(g, kf, l).astype(np.float32))


# ------------------------------------------------------------ association

def test_correspondences_identity_bit_exact(gpu_lib, ctx, c0_surfels):
    _, scan = c0_surfels
    g = lidar_geom(64, 512)
    idx, inl = gpu_lib.correspondences(ctx, g, _t(scan), g, _t(scan), np.eye(4))
    oi, oin = O.correspondences(g, scan, g, scan, np.eye(4))
    assert np.array_equal(_np(idx), oi)
    assert np.array_equal(_np(inl).astype(bool), oin)
    valid = _normal_mask(scan) & (scan[..., 3] > 0)
    I, J = np.meshgrid(np.arange(g.rows), np.arange(g.cols), indexing="ij")
    assert np.array_equal(_np(idx)[valid], (I * g.cols + J)[valid])


def test_correspondences_moved_pose(gpu_lib, ctx, c0, c0_surfels):
    kf, scan = c0_surfels
    g = c0["geom"]
    T = c0["T_gt"]
    idx, inl = gpu_lib.correspondences(ctx, g, _t(scan), g, _t(kf), T)
    oi, oin = O.correspondences(g, scan, g, kf, T)
    mism = int(((_np(idx) != oi) | (_np(inl).astype(bool) != oin)).sum())
    assert mism <= 2e-3 * g.rows * g.cols, mism
    assert oin.sum() > 0.8 * g.rows * g.cols


def test_projection_matches_oracle(gpu_lib, ctx):
    """GPU spherical projection (FP32, own arctangent) against the FP64 oracle
    on random points: identical pixels except where the exact direction lies
    within 1e-3 pixel of a pixel boundary, and there it is one of the two
    neighbours."""
    import torch
    for rows, cols in ((64, 512), (128, 2048)):
        g = lidar_geom(rows, cols)
        rng = np.random.default_rng(rows)
        q = rng.normal(size=(200000, 3))
        q[:, 2] *= 0.3
        q *= rng.uniform(0.5, 49, size=(len(q), 1))
        q32 = q.astype(np.float32)
        gi, gj = gpu_lib.project_points(ctx, g, torch.from_numpy(q32).cuda())
        gi, gj = _np(gi), _np(gj)
        oi, oj, ok = O.project(g, q32.astype(np.float64))
        el = np.arctan2(q32[:, 2].astype(np.float64), np.hypot(q32[:, 0], q32[:, 1]))
        az = np.arctan2(q32[:, 1].astype(np.float64), q32[:, 0].astype(np.float64)) % (2 * np.pi)
        fi = (g.el_top - el) / g.d_el
        fj = az * cols / (2 * np.pi)
        near = (np.abs(fi - np.floor(fi) - 0.5) < 1e-3) | (np.abs(fj - np.floor(fj) - 0.5) < 1e-3)
        assert np.array_equal((gi >= 0), ok) or ((gi >= 0) != ok)[~near].sum() == 0
        same = ok & (gi >= 0) & ~near
        assert np.array_equal(gi[same], oi[same]) and np.array_equal(gj[same], oj[same])
        diff = ok & (gi >= 0) & ((gi != oi) | (gj != oj))
        assert (np.abs(gi[diff] - oi[diff]) <= 1).all()
        dj = np.abs(gj[diff] - oj[diff])
        assert (np.minimum(dj, cols - dj) <= 1).all()
        assert diff.sum() <= near.sum()


# --------------------------------------------------------- normal equations

@pytest.mark.parametrize("prec", [0, 1, 2])
def test_normal_equations_fixed_pose(gpu_lib, ctx, c0, c0_surfels, prec):
    kf, scan = c0_surfels
    g = c0["geom"]
    T = c0["T_gt"] @ O.exp_se3([0.003, -0.002, 0.001, 0.02, 0.01, -0.01])
    neq = gpu_lib.read_neq(gpu_lib.normal_equations(ctx, g, _t(scan), g, _t(kf), T, precision=prec))
    # the oracle on the pixels whose correspondence the GPU shares
    ref = O.normal_equations(g, scan, g, kf, T)
    idx, inl = gpu_lib.correspondences(ctx, g, _t(scan), g, _t(kf), T)
    oi, oin = O.correspondences(g, scan, g, kf, T)
    mism = int(((_np(idx) != oi) | (_np(inl).astype(bool) != oin)).sum())
    assert abs(neq["inliers"] - ref["inliers"]) <= mism
    assert neq["valid"] == ref["valid"]
    A = O.sym6(neq["JtJ"])
    Ar = ref["A"]
    scale = np.sqrt(np.outer(np.diag(Ar), np.diag(Ar)))
    rel = np.abs(A - Ar) / scale
    tol = 1e-5 + 2.0 * mism / max(ref["inliers"], 1)
    assert rel.max() < tol, (rel.max(), mism)
    bscale = np.sqrt(np.diag(Ar) * ref["sum_r2"])
    assert (np.abs(neq["Jtr"] - ref["b"]) / bscale).max() < tol


# ------------------------------------------------------------- registration

def _register_both(gpu_lib, ctx, g, kf, scan, init, p_gpu, p_orc):
    res = gpu_lib.read_result(gpu_lib.register_scan(ctx, g, _t(scan), g, _t(kf), init, p_gpu))
    ref = O.register(g, scan, g, kf, init, p_orc)
    return res, ref


def test_register_config0_matches_oracle(gpu_lib, ctx, c0, c0_surfels):
    kf, scan = c0_surfels
    g = c0["geom"]
    res, ref = _register_both(gpu_lib, ctx, g, kf, scan, np.eye(4), gpu_lib.IcpParams(), O.IcpParams())
    rot, tr = synth.pose_error(res["T"], ref["T"])
    print(f"config0 GPU vs oracle: {rot:.3e} rad {tr:.3e} m; inliers {res['inliers']} vs {ref['inliers']}; "
          f"truncated cost {res['trunc_cost']:.6f} vs {ref['trunc_cost']:.6f}")
    assert res["status"] == ref["status"] == 0
    assert res["iters_run"] == ref["iters_run"] == 20
    assert rot < ROT_TOL and tr < TR_TOL, (rot, tr)
    assert abs(res["inliers"] - ref["inliers"]) <= 2e-3 * ref["valid"]
    # the quality block at the two final poses
    mism = quality_mismatches(gpu_lib, ctx, g, scan, kf, res["T"], ref["T"])
    rr = O.residuals(g, scan, g, kf, ref["T"])
    dr = pose_displacement_bound(res["T"], ref["T"], float(scan[..., 3].max()))
    assert_quality_close(res, ref, mism, 0.5, dr, float(np.abs(rr["r"][rr["inlier"]]).sum()))


@pytest.mark.parametrize("case", ["truth", "perturbed", "self", "far"])
def test_quality_fixed_pose_matches_oracle(gpu_lib, ctx, c0, c0_surfels, case):
    """The quality block alone (a registration with no iterations evaluates it
    at its start pose) at the same pose on both sides: inlier ratio, rms and
    truncated cost within what the counted correspondence mismatches allow."""
    kf, scan = c0_surfels
    g = c0["geom"]
    T = {"truth": c0["T_gt"], "perturbed": c0["T_gt"] @ O.exp_se3([0.01, -0.004, 0.002, 0.08, -0.05, 0.02]),
         "self": np.eye(4), "far": se3(np.eye(3), [0.0, 0.0, 40.0])}[case]
    if case == "self":
        kf = scan
    p = dict(levels=3, iters=(0, 0, 0), d_max=(0.5, 1.0, 2.0))
    res, ref = _register_both(gpu_lib, ctx, g, kf, scan, T, gpu_lib.IcpParams(**p), O.IcpParams(**p))
    assert res["iters_run"] == ref["iters_run"] == 0
    assert np.array_equal(res["T"], T)
    mism = quality_mismatches(gpu_lib, ctx, g, scan, kf, T, T)
    print(f"{case}: inliers {res['inliers']} / {ref['inliers']}, truncated cost {res['trunc_cost']:.6f} / "
          f"{ref['trunc_cost']:.6f}, rms {res['rms']:.6e} / {ref['rms']:.6e}, mismatches {mism}")
    assert_quality_close(res, ref, mism, 0.5)
    if case == "self":
        assert mism == 0 and res["rms"] == 0.0 and res["trunc_cost"] == ref["trunc_cost"]
    if case == "far":
        assert res["inliers"] == 0 and res["trunc_cost"] == ref["trunc_cost"] == 0.25 * ref["valid"]


def test_register_f64_mode_matches_oracle(gpu_lib, ctx, c0, c0_surfels):
    kf, scan = c0_surfels
    g = c0["geom"]
    res, ref = _register_both(gpu_lib, ctx, g, kf, scan, np.eye(4), gpu_lib.IcpParams(precision=2), O.IcpParams())
    rot, tr = synth.pose_error(res["T"], ref["T"])
    print(f"config0 FP64-accumulation vs oracle: {rot:.3e} rad {tr:.3e} m")
    assert rot < ROT_TOL and tr < TR_TOL


def test_register_f32_mode_close(gpu_lib, ctx, c0, c0_surfels):
    kf, scan = c0_surfels
    g = c0["geom"]
    res, ref = _register_both(gpu_lib, ctx, g, kf, scan, np.eye(4), gpu_lib.IcpParams(precision=1), O.IcpParams())
    rot, tr = synth.pose_error(res["T"], ref["T"])
    print(f"config0 pure-FP32 vs oracle: {rot:.3e} rad {tr:.3e} m")
    assert rot < 1e-4 and tr < 1e-4


def test_normal_equations_alternating_poses_repeat_exactly(gpu_lib, ctx, c0, c0_surfels):
    """Reductions at two poses, interleaved: each pose gives bitwise the same
    sums every time (nothing of the previous launch leaks into the next), and
    at the identity against itself J^T r is exactly 0."""
    kf, scan = c0_surfels
    g = c0["geom"]
    poses = [c0["T_gt"], c0["T_gt"] @ O.exp_se3([0.01, 0.0, 0.0, 0.1, 0.0, 0.0])]
    seen = [None, None]
    for rep in range(3):
        for k, T in enumerate(poses):
            r = gpu_lib.read_neq(gpu_lib.normal_equations(ctx, g, _t(scan), g, _t(kf), T))
            vec = np.concatenate([r["JtJ"], r["Jtr"], [r["sum_r2"], r["inliers"]]])
            if seen[k] is None:
                seen[k] = vec
            assert np.array_equal(vec, seen[k]), (rep, k)
        z = gpu_lib.read_neq(gpu_lib.normal_equations(ctx, g, _t(scan), g, _t(scan), np.eye(4)))
        assert (z["Jtr"] == 0.0).all() and z["sum_r2"] == 0.0
    assert not np.array_equal(seen[0], seen[1])


def test_register_zero_residual_identity(gpu_lib, ctx, c0_surfels):
    _, scan = c0_surfels
    g = lidar_geom(64, 512)
    res = gpu_lib.read_result(gpu_lib.register_scan(ctx, g, _t(scan), g, _t(scan), np.eye(4)))
    assert np.array_equal(res["T"], np.eye(4))
    assert res["rms"] == 0.0 and (res["Jtr"] == 0.0).all()


def test_register_deterministic(gpu_lib, ctx, c0_surfels):
    kf, scan = c0_surfels
    g = lidar_geom(64, 512)
    a = gpu_lib.read_result(gpu_lib.register_scan(ctx, g, _t(scan), g, _t(kf), np.eye(4)))
    b = gpu_lib.read_result(gpu_lib.register_scan(ctx, g, _t(scan), g, _t(kf), np.eye(4)))
    assert np.array_equal(a["T"], b["T"]) and np.array_equal(a["JtJ"], b["JtJ"])


def test_exact_recovery_analytic_room_gpu(gpu_lib, ctx):
    c = W.config0(noise=0.0, with_boxes=False, want_normals=True)
    g = c["geom"]

    def surf(r, n):
        s = np.zeros(r.shape + (4,), np.float32)
        s[..., :3] = n
        s[..., 3] = r
        return s

    kf, scan = surf(c["kf"], c["kf_normals"]), surf(c["scan"], c["scan_normals"])
    res = gpu_lib.read_result(gpu_lib.register_scan(ctx, g, _t(scan), g, _t(kf), np.eye(4)))
    rot, tr = synth.pose_error(res["T"], c["T_gt"])
    print(f"analytic room GPU vs truth: {rot:.3e} rad {tr:.3e} m")
    assert rot < ROT_TOL and tr < TR_TOL


def test_register_coarse_to_fine_128x1024(gpu_lib, ctx):
    c = W.config0(rows=128, cols=1024)
    g = c["geom"]
    kf = O.panorama_normals(g, c["kf"]).astype(np.float32)
    scan = O.panorama_normals(g, c["scan"]).astype(np.float32)
    p = dict(levels=3, iters=(10, 10, 10))
    res, ref = _register_both(gpu_lib, ctx, g, kf, scan, np.eye(4), gpu_lib.IcpParams(**p), O.IcpParams(**p))
    rot, tr = synth.pose_error(res["T"], ref["T"])
    print(f"128x1024 3-level GPU vs oracle: {rot:.3e} rad {tr:.3e} m")
    assert res["iters_run"] == ref["iters_run"] == 30
    assert rot < ROT_TOL and tr < TR_TOL, (rot, tr)


def test_register_stop_criterion(gpu_lib, ctx, c0, c0_surfels):
    kf, scan = c0_surfels
    g = c0["geom"]
    p = dict(levels=2, iters=(30, 30), stop_update_norm=1e-6)
    res, ref = _register_both(gpu_lib, ctx, g, kf, scan, np.eye(4), gpu_lib.IcpParams(**p), O.IcpParams(**p))
    assert res["status"] == ref["status"]
    assert abs(res["iters_run"] - ref["iters_run"]) <= 2
    rot, tr = synth.pose_error(res["T"], ref["T"])
    assert rot < ROT_TOL and tr < TR_TOL


def test_failure_no_inliers_and_degenerate(gpu_lib, ctx):
    g = lidar_geom(64, 512)
    zero = np.zeros((64, 512, 4), np.float32)
    res = gpu_lib.read_result(gpu_lib.register_scan(ctx, g, _t(zero), g, _t(zero), np.eye(4)))
    assert res["status"] == 3 and res["iters_run"] == 0 and res["valid"] == 0
    # a single plane: rank-3 normal equations
    el = g.el_top - np.arange(g.rows) * g.d_el
    az = 2 * np.pi * np.arange(g.cols) / g.cols
    E, A = np.meshgrid(el, az, indexing="ij")
    U = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1)
    den = -U[..., 2]
    r = np.where(den > 0.05, 1.5 / np.where(den > 0, den, 1), 0.0)
    r[r > 50] = 0
    s = np.zeros((64, 512, 4), np.float32)
    s[..., 3] = r
    s[r > 0, 2] = 1.0
    init = se3(rot_z(0.01), [0.02, 0.0, 0.0])
    res = gpu_lib.read_result(gpu_lib.register_scan(ctx, g, _t(s), g, _t(s), init))
    assert res["status"] == 2 and res["iters_run"] == 0
    assert np.array_equal(res["T"], init)


def test_invalid_args_raise(gpu_lib, ctx, c0_surfels, torch_mod):
    kf, scan = c0_surfels
    g = lidar_geom(64, 512)
    bad = synth.Geom(64, 500, g.el_top, g.d_el)
    with pytest.raises(gpu_lib.UpsError):
        gpu_lib.register_scan(ctx, bad, _t(scan), g, _t(kf), np.eye(4))
    with pytest.raises(gpu_lib.UpsError):
        gpu_lib.register_scan(ctx, g, _t(scan), g, _t(kf), np.eye(4), gpu_lib.IcpParams(levels=5))
    with pytest.raises(gpu_lib.UpsError):
        gpu_lib.register_scan(ctx, g, _t(scan), g, _t(kf), np.eye(4), gpu_lib.IcpParams(precision=7))
    big = synth.Geom(1024, 4096, g.el_top, g.d_el / 16)
    with pytest.raises(gpu_lib.UpsError):
        d = torch_mod.zeros((1024, 4096), dtype=torch_mod.float32, device="cuda")
        gpu_lib.panorama_normals(ctx, big, d)


# ------------------------------------------------------------------- fusion

def test_fuse_parity(gpu_lib, ctx, c0, c0_surfels, torch_mod):
    kf, scan = c0_surfels
    g = c0["geom"]
    cnt = np.where(_normal_mask(kf) & (kf[..., 3] > 0), 3, 0).astype(np.uint16)
    cnt[::7, ::5] = 0  # some empty keyframe pixels to fill
    kf_in = kf.copy()
    kf_in[cnt == 0] = 0.0
    T = c0["T_gt"]
    kf_d = _t(kf_in)
    cnt_d = _t(cnt.view(np.int16))
    gpu_lib.fuse_scan(ctx, g, _t(scan), g, kf_d, cnt_d, T)
    kg, cg = _np(kf_d), _np(cnt_d).view(np.uint16)
    ko, co = O.fuse(g, scan, g, kf_in, cnt, T)
    mism = int((cg != co).sum())
    assert mism <= 2e-3 * cnt.size, mism
    same = (cg == co) & (co > 0)
    assert same.sum() > 0.8 * cnt.size
    dr = np.abs(kg[..., 3][same] - ko[..., 3][same]) / ko[..., 3][same]
    assert dr.max() < 1e-5, dr.max()
    dn = np.linalg.norm(kg[same][:, :3] - ko[same][:, :3], axis=-1)
    assert dn.max() < 1e-4, dn.max()
    filled = (cnt == 0) & (co == 1)
    assert filled.sum() > 100


def test_fuse_twice_matches_oracle(gpu_lib, ctx, c0, c0_surfels):
    """Two fusions in a row into an initially empty keyframe (the first fills
    it, the second updates it and fills what is still empty): the fill keys
    must be clean for the second call."""
    kf, scan = c0_surfels
    g = c0["geom"]
    T = c0["T_gt"]
    kf_d = _t(np.zeros_like(kf))
    cnt_d = _t(np.zeros(g.shape, np.int16))
    ko = np.zeros(kf.shape)
    co = np.zeros(g.shape, np.uint16)
    for src, pose in ((kf, np.eye(4)), (scan, T)):
        gpu_lib.fuse_scan(ctx, g, _t(src), g, kf_d, cnt_d, pose)
        ko, co = O.fuse(g, src, g, ko, co, pose)
    cg = _np(cnt_d).view(np.uint16)
    mism = int((cg != co).sum())
    assert mism <= 2e-3 * cg.size, mism
    assert (co == 2).sum() > 0.5 * cg.size
    same = (cg == co) & (co > 0)
    kg = _np(kf_d)
    dr = np.abs(kg[..., 3][same] - ko[..., 3][same]) / ko[..., 3][same]
    assert dr.max() < 1e-5
