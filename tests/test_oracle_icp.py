"""Pins of the oracle's registration (Section III-B, Equation 1).

* residual r = (T s2 - s1).N(s1): equals the signed plane offset on planes;
  zero for every pixel when a scan is registered against itself at T = I.
* Jacobian: central finite differences of the oracle's own residuals under
  T <- Exp(delta e_k) T at unchanged correspondences.
* normal equations: equal numpy's J^T J / J^T r on the stacked per-pixel rows,
  symmetric and positive semi-definite.
* 6x6 solve: scipy's Cholesky solve; rank deficiency is reported.
* Exp: scipy.linalg.expm of the 4x4 twist matrix.
* exact recovery: on the analytic box room with exact normals and FP64 ranges,
  Gauss-Newton from the identity returns the true motion to 1e-10.
* projective correspondences: brute-force nearest-pixel search on 8x32.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import synth
from synth import Geom, lidar_geom, se3, rot_x, rot_y, rot_z
from synth import workloads as W

DEG = math.pi / 180


def _hat(w):
    return np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])


def _twist_matrix(xi):
    M = np.zeros((4, 4))
    M[:3, :3] = _hat(xi[:3])
    M[:3, 3] = xi[3:]
    return M


@pytest.mark.parametrize("theta", [0.0, 1e-9, 1e-6, 9.99e-5, 1.001e-4, 1e-3, 0.1, 1.0, 3.0])
def test_exp_matches_expm(theta):
    rng = np.random.default_rng(int(theta * 1e6) % 1000)
    w = rng.normal(size=3)
    w = w / np.linalg.norm(w) * theta
    v = rng.normal(size=3)
    xi = np.concatenate([w, v])
    T = O.exp_se3(xi)
    ref = scipy.linalg.expm(_twist_matrix(xi))
    np.testing.assert_allclose(T, ref, atol=2e-15 * max(1.0, np.abs(v).max() * 4))


def test_compose_is_matrix_product():
    rng = np.random.default_rng(0)
    A = O.exp_se3(rng.normal(size=6))
    B = O.exp_se3(rng.normal(size=6))
    np.testing.assert_allclose(O.compose(A, B), A @ B, atol=1e-14)


def test_solve6_matches_cholesky():
    rng = np.random.default_rng(1)
    M = rng.normal(size=(40, 6)) * np.array([30, 30, 30, 1, 1, 1])
    A = M.T @ M
    b = rng.normal(size=6)
    A21 = np.array([A[a, c] for a in range(6) for c in range(a, 6)])
    st, xi = O.solve6(A21, b)
    assert st == 0
    ref = -scipy.linalg.cho_solve(scipy.linalg.cho_factor(A), b)
    np.testing.assert_allclose(xi, ref, rtol=1e-12, atol=1e-14)


def test_solve6_rank_deficient():
    rng = np.random.default_rng(2)
    M = rng.normal(size=(40, 6))
    M[:, 4] = M[:, 3]                      # two identical columns: rank 5
    A = M.T @ M
    A21 = np.array([A[a, c] for a in range(6) for c in range(a, 6)])
    st, _ = O.solve6(A21, np.ones(6))
    assert st == 2
    st, _ = O.solve6(np.zeros(21), np.ones(6))
    assert st == 2


def _analytic_room(rows=64, cols=512, with_boxes=False):
    """Noise-free room, FP64 ranges, surfels built from the renderer's exact
    face normals (no estimated normals)."""
    c = W.config0(rows=rows, cols=cols, noise=0.0, with_boxes=with_boxes, want_normals=True, dtype=np.float64)
    g = c["geom"]

    def surf(r, n):
        s = np.zeros(r.shape + (4,))
        s[..., :3] = n
        s[..., 3] = r
        return s

    return c, g, surf(c["kf"], c["kf_normals"]), surf(c["scan"], c["scan_normals"])


def test_exact_recovery_analytic_room():
    c, g, kf, scan = _analytic_room()
    res = O.register(g, scan, g, kf, np.eye(4), O.IcpParams(levels=1, iters=(20,)))
    rot, tr = synth.pose_error(res["T"], c["T_gt"])
    assert rot < 1e-10 and tr < 1e-10, (rot, tr)
    # at the recovered pose every inlier lies exactly on its plane
    assert res["rms"] < 1e-9
    # and the final correspondence set is a fixed point: J^T r = 0
    assert np.abs(res["Jtr"]).max() < 1e-6


def test_exact_recovery_coarse_to_fine():
    c, g, kf, scan = _analytic_room(128, 1024)
    p = O.IcpParams(levels=3, iters=(10, 10, 10))
    res = O.register(g, scan, g, kf, np.eye(4), p)
    rot, tr = synth.pose_error(res["T"], c["T_gt"])
    assert rot < 1e-10 and tr < 1e-10, (rot, tr)
    assert res["iters_run"] == 30 and res["status"] == 0


def test_zero_residual_at_identity():
    c = W.config0()
    g = c["geom"]
    s = O.panorama_normals(g, c["scan"])
    res = O.residuals(g, s, g, s, np.eye(4))
    has = (np.abs(s[..., :3]).sum(-1) > 0) & (s[..., 3] > 0)
    I, J = np.meshgrid(np.arange(g.rows), np.arange(g.cols), indexing="ij")
    assert np.array_equal(res["kf_index"][has], (I * g.cols + J)[has])
    assert res["inlier"][has].all()
    assert (res["r"] == 0.0).all()
    ne = O.normal_equations(g, s, g, s, np.eye(4))
    assert (ne["b"] == 0.0).all()
    r = O.register(g, s, g, s, np.eye(4))
    assert np.array_equal(r["T"], np.eye(4))


def test_residual_is_plane_offset():
    """Translating a planar scene's scan by delta along the wall normal gives
    r = delta on that wall (sign and meaning of Equation 1's term)."""
    c, g, kf, scan = _analytic_room()
    delta = 0.013
    # the wall x = +10 has sensor-facing normal (-1, 0, 0)
    n = np.array([-1.0, 0.0, 0.0])
    T = se3(np.eye(3), delta * n)
    res = O.residuals(g, kf, g, kf, T, d_max=0.5)
    on_wall = (np.abs(kf[..., :3] - n).sum(-1) < 1e-12) & res["inlier"]
    assert on_wall.sum() > 500
    np.testing.assert_allclose(res["r"][on_wall], delta, atol=1e-12)


def test_jacobian_finite_differences():
    c = W.config0()
    g = c["geom"]
    kf = O.panorama_normals(g, c["kf"])
    scan = O.panorama_normals(g, c["scan"])
    T = c["T_gt"] @ O.exp_se3([0.002, -0.001, 0.003, 0.01, -0.02, 0.005])
    base = O.residuals(g, scan, g, kf, T)
    h = 1e-6
    checked = 0
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        rp = O.residuals(g, scan, g, kf, O.exp_se3(e) @ T)
        rm = O.residuals(g, scan, g, kf, O.exp_se3(-e) @ T)
        same = base["inlier"] & rp["inlier"] & rm["inlier"] & (rp["kf_index"] == base["kf_index"]) & (
            rm["kf_index"] == base["kf_index"])
        fd = (rp["r"] - rm["r"]) / (2 * h)
        Jk = base["J"][..., k]
        scale = np.abs(Jk[same]).max()
        err = np.abs(fd[same] - Jk[same]).max()
        assert err < 1e-7 * scale + 1e-8, (k, err, scale)
        checked += same.sum()
    assert checked > 6 * 10000


def test_normal_equations_match_stacked_rows():
    c = W.config0()
    g = c["geom"]
    kf = O.panorama_normals(g, c["kf"])
    scan = O.panorama_normals(g, c["scan"])
    T = c["T_gt"] @ O.exp_se3([0.01, 0.0, -0.01, 0.05, 0.0, 0.02])
    res = O.residuals(g, scan, g, kf, T)
    Js = res["J"][res["inlier"]]
    rs = res["r"][res["inlier"]]
    ne = O.normal_equations(g, scan, g, kf, T)
    np.testing.assert_allclose(ne["A"], Js.T @ Js, rtol=1e-10)
    np.testing.assert_allclose(ne["b"], Js.T @ rs, rtol=1e-9, atol=1e-9)
    assert ne["inliers"] == res["inlier"].sum()
    assert ne["valid"] == (scan[..., 3] > 0).sum()
    np.testing.assert_allclose(ne["sum_r2"], (rs ** 2).sum(), rtol=1e-12)
    A = ne["A"]
    assert np.array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() >= -1e-12 * np.trace(A)


def _brute_rays(g):
    el = g.el_top - np.arange(g.rows) * g.d_el
    az = 2 * np.pi * np.arange(g.cols) / g.cols
    E, A = np.meshgrid(el, az, indexing="ij")
    return np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1)


def test_correspondences_brute_force_8x32():
    """For every scan pixel: transform its point with numpy, find the nearest
    keyframe pixel by exhaustive angular search, then apply the distance and
    normal gates."""
    g = Geom(8, 32, math.radians(12.0), math.radians(24.0) / 7, 0.0, 50.0)
    rng = np.random.default_rng(4)
    U = _brute_rays(g)

    def rand_surf():
        s = np.zeros((8, 32, 4))
        s[..., 3] = rng.uniform(3.0, 6.0, size=(8, 32))
        n = -U + rng.normal(size=U.shape) * 0.4
        n /= np.linalg.norm(n, axis=-1, keepdims=True)
        s[..., :3] = n
        s[rng.random((8, 32)) < 0.1, :3] = 0.0
        s[rng.random((8, 32)) < 0.05, 3] = 0.0
        return s

    kf, scan = rand_surf(), rand_surf()
    T = se3(rot_z(0.05) @ rot_x(0.02), [0.1, -0.05, 0.02])
    d_max, cos_t = 1.0, math.cos(math.radians(40))
    idx, inl = O.correspondences(g, scan, g, kf, T, d_max, cos_t)
    R, t = T[:3, :3], T[:3, 3]
    el_rows = g.el_top - np.arange(8) * g.d_el
    az_cols = 2 * np.pi * np.arange(32) / 32
    n_inl = 0
    for i in range(8):
        for j in range(32):
            s2 = scan[i, j]
            if not (s2[3] > 0 and np.abs(s2[:3]).sum() > 0):
                assert idx[i, j] == -1 and not inl[i, j]
                continue
            q = R @ (s2[3] * U[i, j]) + t
            el = math.atan2(q[2], math.hypot(q[0], q[1]))
            az = math.atan2(q[1], q[0]) % (2 * math.pi)
            ki = int(np.argmin(np.abs(el_rows - el)))
            kj = int(np.argmin(np.abs((az_cols - az + math.pi) % (2 * math.pi) - math.pi)))
            if abs(el_rows[ki] - el) > g.d_el / 2:
                assert idx[i, j] == -1
                continue
            assert idx[i, j] == ki * 32 + kj
            s1 = kf[ki, kj]
            ok = s1[3] > 0 and np.abs(s1[:3]).sum() > 0
            if ok:
                x1 = s1[3] * U[ki, kj]
                ok = np.linalg.norm(q - x1) <= d_max and (R @ s2[:3]) @ s1[:3] >= cos_t
            assert bool(inl[i, j]) == bool(ok), (i, j)
            n_inl += ok
    assert n_inl > 20


def test_degenerate_single_plane():
    """A single plane constrains only 3 of 6 DoF: DEGENERATE, pose unchanged."""
    g = lidar_geom(64, 512)
    U = _brute_rays(g)
    n = np.array([0.0, 0.0, 1.0])
    den = U @ (-n)
    r = np.where(den > 0.05, 1.5 / np.where(den > 0, den, 1), 0.0)
    r[r > g.r_max] = 0
    s = np.zeros((64, 512, 4))
    s[..., 3] = r
    s[r > 0, :3] = n
    init = se3(rot_z(0.01), [0.02, 0.0, 0.0])
    res = O.register(g, s, g, s, init)
    assert res["status"] == 2
    np.testing.assert_array_equal(res["T"], init)
    assert res["iters_run"] == 0


def test_no_inliers():
    g = lidar_geom(64, 512)
    s = np.zeros((64, 512, 4))
    res = O.register(g, s, g, s, np.eye(4))
    assert res["status"] == 3 and res["valid"] == 0 and res["inlier_ratio"] == 0.0


def test_register_config0_converges_near_truth():
    c = W.config0()
    g = c["geom"]
    kf = O.panorama_normals(g, c["kf"])
    scan = O.panorama_normals(g, c["scan"])
    res = O.register(g, scan, g, kf, np.eye(4))
    rot, tr = synth.pose_error(res["T"], c["T_gt"])
    assert rot < 2e-4 and tr < 5e-3, (rot, tr)
    assert res["inlier_ratio"] > 0.9
    # converged: the normal equations at the final pose have J^T r ~ 0 relative
    # to their scale
    A = O.sym6(res["JtJ"])
    step = np.linalg.solve(A, res["Jtr"])
    assert np.abs(step).max() < 1e-6
