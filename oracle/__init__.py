"""FP64 CPU oracle for the UPSLAM registration path -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  The product library
(``paper_2101_00585_amd``) never imports, links or calls it, and the two share
no code: the oracle is plain single-threaded C (``orc.c``, compiled with gcc
-O2 -fno-fast-math) plus numpy marshalling here.

Each function follows a passage of the paper (arXiv 2101.00585):

* normals by the cross product of two image-neighbour vectors, smoothed by an
  edge-aware a-trous filter -- Section III-A (Data Intake);
* projective correspondences, the similarity filter Omega_{d,theta} and the
  point-to-plane error of Equation 1 -- Section III-B (Motion Estimation);
* registration quality as inliers over valid ranges and the count-weighted
  keyframe update saturated at 10 -- Section III-C (Keyframe Update).

Where the paper gives no value or detail the reading is stated next to the
function and in the defaults below.  Pins: tests/test_oracle_*.py.

Parity unpinned: the exact weights of the a-trous filter (the paper names the
filter but gives no taps, scales or number of levels).  Its invariants and
its wide-sigma limit, a plain B3-spline convolution, are pinned; the weights
themselves follow the stated reading only.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STATUS = {0: "CONVERGED", 1: "MAX_ITERS", 2: "DEGENERATE", 3: "NO_INLIERS", 4: "FALLBACK_USED"}


# UPS_SANITIZE=1 selects a build instrumented with AddressSanitizer and
# UBSan (clang; its runtime must be preloaded into the process, see
# tests/run_cpu_sanitized.sh)
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined", "-shared-libsan"]


def sanitized() -> bool:
    return os.environ.get("UPS_SANITIZE") == "1"


def _so_path(sanitize):
    return os.path.join(_HERE, "liboracle_san.so" if sanitize else "liboracle.so")


def build(sanitize: bool | None = None) -> str:
    sanitize = sanitized() if sanitize is None else sanitize
    so = _so_path(sanitize)
    tmp = so + ".tmp%d" % os.getpid()
    if sanitize:
        cmd = ["/opt/rocm/llvm/bin/clang", "-std=c11", *SANITIZE_FLAGS]
    else:
        cmd = ["gcc", "-std=c11", "-O2"]
    subprocess.check_call(cmd + ["-fno-fast-math", "-fPIC", "-shared", "-o", tmp, os.path.join(_HERE, "orc.c"), "-lm"])
    os.replace(tmp, so)
    return so


def _lib():
    global _LIB
    if _LIB is None:
        so = _so_path(sanitized())
        srcs = [os.path.join(_HERE, f) for f in ("orc.c", "orc.h")]
        if not os.path.exists(so) or os.path.getmtime(so) < max(os.path.getmtime(s) for s in srcs):
            build()
        _LIB = ctypes.CDLL(so)
        for name in ("orc_project", "orc_raw_normals", "orc_atrous", "orc_panorama_normals", "orc_pyramid_level",
                     "orc_residuals", "orc_normal_equations", "orc_normal_equations_irls", "orc_solve6",
                     "orc_register", "orc_fuse", "orc_free_space_violations", "orc_remove_marked",
                     "orc_splat_sweep"):
            getattr(_LIB, name).restype = ctypes.c_int
    return _LIB


# ----------------------------------------------------------------------------
# parameter structs
# ----------------------------------------------------------------------------

class _Geom(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("el_top", ctypes.c_double),
                ("d_el", ctypes.c_double), ("r_min", ctypes.c_double), ("r_max", ctypes.c_double)]


class _NormalParams(ctypes.Structure):
    _fields_ = [("atrous_levels", ctypes.c_int32), ("sigma_n", ctypes.c_double), ("sigma_r", ctypes.c_double),
                ("max_rel_jump", ctypes.c_double)]


class _IcpParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("iters", ctypes.c_int32 * 4), ("d_max", ctypes.c_double * 4),
                ("cos_theta_max", ctypes.c_double), ("stop_update_norm", ctypes.c_double),
                ("min_inliers", ctypes.c_int32), ("irls_delta", ctypes.c_double)]


class _IcpResult(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double * 12), ("rms", ctypes.c_double), ("trunc_cost", ctypes.c_double),
                ("inlier_ratio", ctypes.c_double), ("inliers", ctypes.c_int64), ("valid", ctypes.c_int64),
                ("iters_run", ctypes.c_int32), ("status", ctypes.c_int32), ("level_iters", ctypes.c_int32 * 4),
                ("JtJ", ctypes.c_double * 21),
                ("Jtr", ctypes.c_double * 6), ("last_update_norm", ctypes.c_double)]


class _ConsistencyParams(ctypes.Structure):
    _fields_ = [("margin_abs", ctypes.c_double), ("margin_rel", ctypes.c_double), ("min_count", ctypes.c_int32)]


class _FuseParams(ctypes.Structure):
    _fields_ = [("d_max", ctypes.c_double), ("cos_theta_max", ctypes.c_double),
                ("min_cos_incidence", ctypes.c_double), ("max_count", ctypes.c_int32)]


@dataclass
class NormalParams:
    """Readings for Section III-A: two a-trous levels, sigma_n = 0.5,
    sigma_r = 0.05 (relative), occlusion cut at a 50 % range jump."""
    atrous_levels: int = 2
    sigma_n: float = 0.5
    sigma_r: float = 0.05
    max_rel_jump: float = 0.5

    def _c(self):
        return _NormalParams(self.atrous_levels, self.sigma_n, self.sigma_r, self.max_rel_jump)


@dataclass
class IcpParams:
    """Readings for Section III-B: d_max = 0.5 m at level 0 doubling per
    coarser level, theta_max = 30 deg, at least 64 inliers.  ``irls_delta``
    0 minimises the squared residuals; > 0 minimises the absolute residuals of
    Equation 1 by reweighting with 1 / max(|r|, irls_delta)."""
    levels: int = 1
    iters: tuple = (20, 0, 0, 0)
    d_max: tuple = (0.5, 1.0, 2.0, 4.0)
    cos_theta_max: float = math.cos(math.radians(30.0))
    stop_update_norm: float = 0.0
    min_inliers: int = 64
    irls_delta: float = 0.0

    def _c(self):
        it = list(self.iters) + [0] * (4 - len(self.iters))
        dm = list(self.d_max) + [self.d_max[-1]] * (4 - len(self.d_max))
        return _IcpParams(self.levels, (ctypes.c_int32 * 4)(*it), (ctypes.c_double * 4)(*dm), self.cos_theta_max,
                          self.stop_update_norm, self.min_inliers, self.irls_delta)


@dataclass
class FuseParams:
    """Readings for Section III-C: 0.2 m distance gate, 30 deg normal gate,
    keyframe rays within ~84 deg of the surface normal, count saturating at 10."""
    d_max: float = 0.2
    cos_theta_max: float = math.cos(math.radians(30.0))
    min_cos_incidence: float = 0.1
    max_count: int = 10

    def _c(self):
        return _FuseParams(self.d_max, self.cos_theta_max, self.min_cos_incidence, self.max_count)


def _geom(g) -> _Geom:
    return _Geom(int(g.rows), int(g.cols), float(g.el_top), float(g.d_el), float(g.r_min), float(g.r_max))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def pose12(T) -> np.ndarray:
    T = np.asarray(T, dtype=np.float64)
    return np.ascontiguousarray(np.concatenate([T[:3, :3].reshape(9), T[:3, 3]]))


def pose44(p12) -> np.ndarray:
    p = np.asarray(p12, dtype=np.float64)
    T = np.eye(4)
    T[:3, :3] = p[:9].reshape(3, 3)
    T[:3, 3] = p[9:12]
    return T


def sym6(A21) -> np.ndarray:
    A = np.zeros((6, 6))
    e = 0
    for a in range(6):
        for c in range(a, 6):
            A[a, c] = A[c, a] = A21[e]
            e += 1
    return A


# ----------------------------------------------------------------------------
# wrappers
# ----------------------------------------------------------------------------

def ray(g, i, j) -> np.ndarray:
    u = (ctypes.c_double * 3)()
    _lib().orc_ray(ctypes.byref(_geom(g)), int(i), int(j), u)
    return np.array(u[:])


def project(g, q):
    """Nearest pixel of each point q [N, 3]; returns (i, j, ok) arrays."""
    q = _f64(q, (-1, 3))
    n = q.shape[0]
    ii = np.full(n, -1, np.int32)
    jj = np.full(n, -1, np.int32)
    ok = np.zeros(n, bool)
    gc = _geom(g)
    L = _lib()
    ci, cj = ctypes.c_int32(), ctypes.c_int32()
    for k in range(n):
        if L.orc_project(ctypes.byref(gc), _ptr(q[k]), ctypes.byref(ci), ctypes.byref(cj)):
            ii[k], jj[k], ok[k] = ci.value, cj.value, True
    return ii, jj, ok


def raw_normals(g, depth, max_rel_jump=0.5) -> np.ndarray:
    d = _f64(depth, (g.rows, g.cols))
    out = np.zeros((g.rows, g.cols, 4))
    _lib().orc_raw_normals(ctypes.byref(_geom(g)), _ptr(d), ctypes.c_double(max_rel_jump), _ptr(out))
    return out


def atrous(g, surfel, levels=2, sigma_r=0.05, sigma_n=0.5) -> np.ndarray:
    s = _f64(surfel, (g.rows, g.cols, 4))
    out = np.zeros_like(s)
    _lib().orc_atrous(ctypes.byref(_geom(g)), _ptr(s), int(levels), ctypes.c_double(sigma_r),
                      ctypes.c_double(sigma_n), _ptr(out))
    return out


def panorama_normals(g, depth, params: NormalParams | None = None) -> np.ndarray:
    p = params or NormalParams()
    d = _f64(depth, (g.rows, g.cols))
    out = np.zeros((g.rows, g.cols, 4))
    pc = p._c()
    _lib().orc_panorama_normals(ctypes.byref(_geom(g)), _ptr(d), ctypes.byref(pc), _ptr(out))
    return out


def pyramid_level(g, surfel, level) -> np.ndarray:
    s = _f64(surfel, (g.rows, g.cols, 4))
    out = np.zeros((g.rows >> level, g.cols >> level, 4))
    _lib().orc_pyramid_level(ctypes.byref(_geom(g)), _ptr(s), int(level), _ptr(out))
    return out


def residuals(sg, scan, kg, kf, T, d_max=0.5, cos_theta_max=math.cos(math.radians(30.0))):
    """Per scan pixel: keyframe index (-1 none), inlier flag, residual r and
    Jacobian row J [N, 6] (zeros for non-inliers)."""
    s = _f64(scan, (sg.rows, sg.cols, 4))
    k = _f64(kf, (kg.rows, kg.cols, 4))
    n = sg.rows * sg.cols
    idx = np.zeros(n, np.int32)
    inl = np.zeros(n, np.uint8)
    r = np.zeros(n)
    J = np.zeros((n, 6))
    _lib().orc_residuals(ctypes.byref(_geom(sg)), _ptr(s), ctypes.byref(_geom(kg)), _ptr(k), _ptr(pose12(T)),
                         ctypes.c_double(d_max), ctypes.c_double(cos_theta_max), _ptr(idx), _ptr(inl), _ptr(r),
                         _ptr(J))
    return dict(kf_index=idx.reshape(sg.rows, sg.cols), inlier=inl.reshape(sg.rows, sg.cols).astype(bool),
                r=r.reshape(sg.rows, sg.cols), J=J.reshape(sg.rows, sg.cols, 6))


def correspondences(sg, scan, kg, kf, T, d_max=0.5, cos_theta_max=math.cos(math.radians(30.0))):
    res = residuals(sg, scan, kg, kf, T, d_max, cos_theta_max)
    return res["kf_index"], res["inlier"]


def normal_equations(sg, scan, kg, kf, T, d_max=0.5, cos_theta_max=math.cos(math.radians(30.0)), irls_delta=0.0):
    """Normal equations at pose T; irls_delta > 0 weights each inlier by
    1 / max(|r|, irls_delta) (the absolute-value objective's IRLS step)."""
    s = _f64(scan, (sg.rows, sg.cols, 4))
    k = _f64(kf, (kg.rows, kg.cols, 4))
    A = np.zeros(21)
    b = np.zeros(6)
    s2 = ctypes.c_double()
    ni, nv = ctypes.c_int64(), ctypes.c_int64()
    _lib().orc_normal_equations_irls(ctypes.byref(_geom(sg)), _ptr(s), ctypes.byref(_geom(kg)), _ptr(k),
                                     _ptr(pose12(T)), ctypes.c_double(d_max), ctypes.c_double(cos_theta_max),
                                     ctypes.c_double(irls_delta), _ptr(A), _ptr(b), ctypes.byref(s2),
                                     ctypes.byref(ni), ctypes.byref(nv))
    return dict(A21=A, A=sym6(A), b=b, sum_r2=s2.value, inliers=ni.value, valid=nv.value)


def solve6(A21, b):
    A21 = _f64(A21, (21,))
    b = _f64(b, (6,))
    xi = np.zeros(6)
    st = _lib().orc_solve6(_ptr(A21), _ptr(b), _ptr(xi))
    return st, xi


def exp_se3(xi) -> np.ndarray:
    xi = _f64(xi, (6,))
    T = np.zeros(12)
    _lib().orc_exp_se3(_ptr(xi), _ptr(T))
    return pose44(T)


def compose(A, B) -> np.ndarray:
    out = np.zeros(12)
    _lib().orc_compose(_ptr(pose12(A)), _ptr(pose12(B)), _ptr(out))
    return pose44(out)


def register(sg, scan, kg, kf, init, params: IcpParams | None = None) -> dict:
    """Coarse-to-fine Gauss-Newton point-to-plane registration of a scan
    surfel image against a keyframe surfel image starting from ``init``
    (scan -> keyframe).  Returns the result fields as a dict."""
    p = params or IcpParams()
    s = _f64(scan, (sg.rows, sg.cols, 4))
    k = _f64(kf, (kg.rows, kg.cols, 4))
    res = _IcpResult()
    pc = p._c()
    _lib().orc_register(ctypes.byref(_geom(sg)), _ptr(s), ctypes.byref(_geom(kg)), _ptr(k), _ptr(pose12(init)),
                        ctypes.byref(pc), ctypes.byref(res))
    return dict(T=pose44(res.T), rms=res.rms, trunc_cost=res.trunc_cost, inlier_ratio=res.inlier_ratio,
                inliers=res.inliers, valid=res.valid, iters_run=res.iters_run, status=res.status,
                level_iters=list(res.level_iters),
                JtJ=np.array(res.JtJ[:]), Jtr=np.array(res.Jtr[:]), last_update_norm=res.last_update_norm)


def fuse(sg, scan, kg, kf, kf_count, T, params: FuseParams | None = None):
    """Fuse a registered scan surfel image into a keyframe; returns the new
    (keyframe surfels, counts) and leaves the inputs untouched."""
    p = params or FuseParams()
    s = _f64(scan, (sg.rows, sg.cols, 4))
    k = _f64(kf, (kg.rows, kg.cols, 4)).copy()
    c = np.ascontiguousarray(np.asarray(kf_count, dtype=np.uint16).reshape(kg.rows, kg.cols)).copy()
    pc = p._c()
    _lib().orc_fuse(ctypes.byref(_geom(sg)), _ptr(s), ctypes.byref(_geom(kg)), _ptr(k), _ptr(c), _ptr(pose12(T)),
                    ctypes.byref(pc))
    return k, c


@dataclass
class ConsistencyParams:
    """Readings for the moving-object check across keyframes (Section III-C):
    a sample is contradicted when the other keyframe saw more than
    max(margin_abs, margin_rel * range) beyond it on every ray of a 3x3
    neighbourhood, each with at least ``min_count`` fused samples."""
    margin_abs: float = 0.2
    margin_rel: float = 0.02
    min_count: int = 1

    def _c(self):
        return _ConsistencyParams(self.margin_abs, self.margin_rel, self.min_count)


def free_space_violations(ga, a, gb, b, b_count, T_ba, params: ConsistencyParams | None = None) -> np.ndarray:
    """Mask [rows_a, cols_a] of keyframe A's samples that keyframe B saw
    through; T_ba maps A's frame into B's.  b_count None: any count votes."""
    p = params or ConsistencyParams()
    sa = _f64(a, (ga.rows, ga.cols, 4))
    sb = _f64(b, (gb.rows, gb.cols, 4))
    cb = None
    if b_count is not None:
        cb = np.ascontiguousarray(np.asarray(b_count, dtype=np.uint16).reshape(gb.rows, gb.cols))
    mask = np.zeros((ga.rows, ga.cols), np.uint8)
    pc = p._c()
    _lib().orc_free_space_violations(ctypes.byref(_geom(ga)), _ptr(sa), ctypes.byref(_geom(gb)), _ptr(sb),
                                     None if cb is None else _ptr(cb), _ptr(pose12(T_ba)), ctypes.byref(pc),
                                     _ptr(mask))
    return mask.astype(bool)


def keyframe_consistency(ga, a, a_count, gb, b, b_count, T_ba, params: ConsistencyParams | None = None):
    """The mutual check: both masks from the unmodified keyframes, then the
    marked samples of each removed.  Returns (a, a_count, b, b_count, mask_a,
    mask_b) as new arrays."""
    mask_a = free_space_violations(ga, a, gb, b, b_count, T_ba, params)
    T = pose44(pose12(T_ba))
    T_ab = np.eye(4)
    T_ab[:3, :3] = T[:3, :3].T
    T_ab[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    mask_b = free_space_violations(gb, b, ga, a, a_count, T_ab, params)
    out = []
    for g, s, c, m in ((ga, a, a_count, mask_a), (gb, b, b_count, mask_b)):
        s2 = _f64(s, (g.rows, g.cols, 4)).copy()
        c2 = None if c is None else np.ascontiguousarray(np.asarray(c, dtype=np.uint16).reshape(g.rows, g.cols)).copy()
        mm = np.ascontiguousarray(m.astype(np.uint8))
        _lib().orc_remove_marked(ctypes.byref(_geom(g)), _ptr(s2), None if c2 is None else _ptr(c2), _ptr(mm))
        out += [s2, c2]
    return out[0], out[1], out[2], out[3], mask_a, mask_b



LOOP_NONE, LOOP_WEAK, LOOP_STRONG = 0, 1, 2


def loop_closure_classes(ratios, statuses, new_keyframe_ratio):
    """Section III-C: a loop-closure registration whose quality (inlier
    ratio) is higher than the threshold for seeking a new keyframe is a strong
    closure (its keyframe becomes the current one); one higher than 75 % of it
    is a weak closure (a pose-graph edge only); registrations that failed
    (status 2 degenerate, 3 too few inliers) close nothing.  Returns the
    classes and the strong closure with the highest ratio (first of equals),
    -1 when there is none."""
    classes = []
    best, best_ratio = -1, None
    for k, (q, st) in enumerate(zip(ratios, statuses)):
        if st in (2, 3):
            c = LOOP_NONE
        elif q > new_keyframe_ratio:
            c = LOOP_STRONG
        elif q > 0.75 * new_keyframe_ratio:
            c = LOOP_WEAK
        else:
            c = LOOP_NONE
        classes.append(c)
        if c == LOOP_STRONG and (best_ratio is None or q > best_ratio):
            best, best_ratio = k, q
    return np.array(classes, dtype=np.int32), best


def splat_sweep(raw_g, raw, col_T, out_g) -> np.ndarray:
    """Panorama of out_g from a sweep (range image of raw_g whose column j
    was measured in the frame that the 4x4 col_T[j] maps into the reference
    frame; None: all identity): nearest range per pixel, 0 where empty."""
    r = _f64(raw, (raw_g.rows, raw_g.cols))
    C = None
    if col_T is not None:
        C = np.ascontiguousarray(np.stack([pose12(T) for T in np.asarray(col_T, np.float64)]))
    out = np.zeros((out_g.rows, out_g.cols))
    _lib().orc_splat_sweep(ctypes.byref(_geom(raw_g)), _ptr(r), None if C is None else _ptr(C),
                           ctypes.byref(_geom(out_g)), _ptr(out))
    return out

