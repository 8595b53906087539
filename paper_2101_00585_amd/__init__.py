"""Python binding of the MI355X projective-ICP library (``libupslam.so``).

Argument marshalling only: every step of the registration path runs in the
HIP kernels behind the C ABI declared in ``include/upslam.h``.  PyTorch
supplies device memory and streams; tensors are passed by ``data_ptr()`` and
work is enqueued on ``torch.cuda.current_stream()``.

The library implements UPSLAM's (arXiv 2101.00585) per-sweep path:
``panorama_normals`` (Section III-A), ``register_scan`` (Section III-B,
Equation 1) and ``fuse_scan`` (Section III-C), plus ``correspondences`` and
``normal_equations`` at a fixed pose and ``pyramid_level``.

There is no CPU fallback: if the shared library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# UPS_SANITIZE=1 loads the build whose host code carries AddressSanitizer and
# UBSan (python -m paper_2101_00585_amd.build --sanitize)
_SO = os.path.join(_HERE, "libupslam_san.so" if os.environ.get("UPS_SANITIZE") == "1" else "libupslam.so")
_LIB = None

STATUS = {0: "CONVERGED", 1: "MAX_ITERS", 2: "DEGENERATE", 3: "NO_INLIERS", 4: "FALLBACK_USED"}
STATUS_CONVERGED, STATUS_MAX_ITERS, STATUS_DEGENERATE, STATUS_NO_INLIERS, STATUS_FALLBACK_USED = range(5)
PREC_KAHAN_F64 = 0
PREC_F32 = 1
PREC_F64 = 2


class UpsError(RuntimeError):
    pass


# ----------------------------------------------------------------------------
# C structs (layouts of include/upslam.h)
# ----------------------------------------------------------------------------

class ups_geom(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("el_top", ctypes.c_double),
                ("d_el", ctypes.c_double), ("r_min", ctypes.c_double), ("r_max", ctypes.c_double)]


class ups_pose(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3)]


class ups_normal_params(ctypes.Structure):
    _fields_ = [("atrous_levels", ctypes.c_int32), ("sigma_n", ctypes.c_float), ("sigma_r", ctypes.c_float),
                ("max_rel_jump", ctypes.c_float)]


class ups_icp_params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("iters", ctypes.c_int32 * 4), ("d_max", ctypes.c_float * 4),
                ("cos_theta_max", ctypes.c_float), ("stop_update_norm", ctypes.c_double),
                ("min_inliers", ctypes.c_int32), ("precision", ctypes.c_int32), ("irls_delta", ctypes.c_float)]


class ups_icp_result(ctypes.Structure):
    _fields_ = [("T", ups_pose), ("rms", ctypes.c_double), ("trunc_cost", ctypes.c_double),
                ("inlier_ratio", ctypes.c_double), ("inliers", ctypes.c_int64), ("valid", ctypes.c_int64),
                ("iters_run", ctypes.c_int32), ("status", ctypes.c_int32), ("level_iters", ctypes.c_int32 * 4),
                ("JtJ", ctypes.c_double * 21),
                ("Jtr", ctypes.c_double * 6), ("last_update_norm", ctypes.c_double)]


class ups_normal_eq(ctypes.Structure):
    _fields_ = [("JtJ", ctypes.c_double * 21), ("Jtr", ctypes.c_double * 6), ("sum_r2", ctypes.c_double),
                ("inliers", ctypes.c_int64), ("valid", ctypes.c_int64)]


class ups_fuse_params(ctypes.Structure):
    _fields_ = [("d_max", ctypes.c_float), ("cos_theta_max", ctypes.c_float),
                ("min_cos_incidence", ctypes.c_float), ("max_count", ctypes.c_int32)]


class ups_batch_item(ctypes.Structure):
    _fields_ = [("scan_g", ups_geom), ("kf_g", ups_geom), ("scan_depth_d", ctypes.c_void_p),
                ("kf_depth_d", ctypes.c_void_p), ("scan_surfel_d", ctypes.c_void_p),
                ("kf_surfel_d", ctypes.c_void_p)]


RESULT_BYTES = ctypes.sizeof(ups_icp_result)
NEQ_BYTES = ctypes.sizeof(ups_normal_eq)

_P = ctypes.c_void_p


def load():
    """Load the built library (``python -m paper_2101_00585_amd.build``)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_SO):
        raise UpsError(f"{_SO} is not built: run `python -m paper_2101_00585_amd.build`")
    lib = ctypes.CDLL(_SO)
    sig = {
        "ups_context_create": [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64],
        "ups_panorama_normals": [_P, _P, _P, _P, _P, _P],
        "ups_pyramid_level": [_P, _P, _P, ctypes.c_int32, _P, _P],
        "ups_register_scan": [_P, _P, _P, _P, _P, _P, _P, _P, _P],
        "ups_register_scan_noalloc": [_P, _P, _P, _P, _P, _P, _P, _P],
        "ups_fuse_scan": [_P, _P, _P, _P, _P, _P, _P, _P, _P],
        "ups_correspondences": [_P, _P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float, _P, _P, _P],
        "ups_register_scan_world": [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
        "ups_correspondences_world": [_P, _P, _P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float, _P, _P, _P],
        "ups_normal_equations": [_P, _P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_float, ctypes.c_int32, _P, _P],
        "ups_project_points": [_P, _P, _P, ctypes.c_int64, _P, _P, _P],
        "ups_batch_create": [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.POINTER(_P)],
        "ups_batch_normals": [_P, _P, _P, _P],
        "ups_register_batch": [_P, _P, _P, _P, _P],
        "ups_register_batch_fallback": [_P, _P, ctypes.c_double, _P, _P],
        "ups_batch_fallback_plan": [_P, _P, ctypes.c_double, _P, _P, _P],
        "ups_batch_fallback_run": [_P, _P, _P, _P],
        "ups_batch_grid_search": [_P, _P, _P, _P, _P, _P, _P, _P],
        "ups_batch_pixels_per_thread": [_P, _P],
        "ups_batch_schedule": [_P, _P, _P],
        "ups_batch_set_scheduler": [_P, ctypes.c_int32],
        "ups_batch_set_iterations": [_P, _P],
        "ups_batch_set_pyramid_mode": [_P, ctypes.c_int32],
        "ups_debug_reverse_tile_order": [ctypes.c_int32],
        "ups_debug_level_spin_limit": [ctypes.c_int64],
        "ups_splat_sweep": [_P, _P, _P, _P, _P, _P, _P],
        "ups_keyframe_consistency": [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P],
        "ups_classify_loop_closures": [_P, ctypes.c_int32, _P, ctypes.c_double, _P, _P, _P],
        "ups_autotune": [_P, ctypes.c_char_p],
        "ups_batch_time_iteration": [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(ctypes.c_float)],
    }
    i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    sig.update({
        "ups_proposal_create": [_P, i32, ctypes.POINTER(_P)],
        "ups_proposal_set_params": [_P, _P, i64],
        "ups_proposal_get_params": [_P, _P, i64],
        "ups_proposal_get_grads": [_P, _P, i64],
        "ups_proposal_save_checkpoint": [_P, ctypes.c_char_p],
        "ups_proposal_load_checkpoint": [_P, ctypes.c_char_p],
        "ups_proposal_activations": [_P, i32, i32, _P, _P],
        "ups_proposal_save": [_P, ctypes.c_char_p],
        "ups_proposal_load": [_P, ctypes.c_char_p],
        "ups_proposal_plan_input": [_P, i32, _P, _P],
        "ups_proposal_input": [_P, _P, _P],
        "ups_proposal_forward": [_P, i32, _P, _P, _P],
        "ups_proposal_poses": [_P, i32, _P, _P, _P],
        "ups_proposal_train_step": [_P, i32, _P, _P, f32, _P, _P],
        "ups_conv3x3_forward": [i32, i32, i32, i32, i32, i32, _P, _P, _P, _P, _P],
        "ups_conv3x3_backward_data": [i32, i32, i32, i32, i32, i32, _P, _P, _P, _P, _P],
        "ups_conv3x3_backward_weight": [i32, i32, i32, i32, i32, i32, _P, _P, _P, _P, _P, _P, i64, _P],
    })
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.ups_proposal_num_params.argtypes = []
    lib.ups_proposal_num_params.restype = ctypes.c_int64
    lib.ups_conv3x3_backward_weight_work.argtypes = [ctypes.c_int32] * 6
    lib.ups_conv3x3_backward_weight_work.restype = ctypes.c_int64
    lib.ups_proposal_destroy.argtypes = [_P]
    lib.ups_proposal_destroy.restype = None
    lib.ups_batch_destroy.argtypes = [_P]
    lib.ups_batch_destroy.restype = None
    lib.ups_context_destroy.argtypes = [_P]
    lib.ups_context_destroy.restype = None
    lib.ups_last_error.argtypes = []
    lib.ups_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _check(rc):
    if rc != 0:
        msg = _LIB.ups_last_error().decode()
        raise UpsError(f"upslam error {rc}: {msg}")


# ----------------------------------------------------------------------------
# parameters
# ----------------------------------------------------------------------------

@dataclass
class NormalParams:
    atrous_levels: int = 2
    sigma_n: float = 0.5
    sigma_r: float = 0.05
    max_rel_jump: float = 0.5

    def c(self):
        return ups_normal_params(self.atrous_levels, self.sigma_n, self.sigma_r, self.max_rel_jump)


@dataclass
class IcpParams:
    levels: int = 1
    iters: tuple = (20, 0, 0, 0)
    d_max: tuple = (0.5, 1.0, 2.0, 4.0)
    cos_theta_max: float = math.cos(math.radians(30.0))
    stop_update_norm: float = 0.0
    min_inliers: int = 64
    precision: int = PREC_KAHAN_F64
    irls_delta: float = 0.0  # > 0: absolute residuals (Equation 1) by IRLS, weights 1 / max(|r|, irls_delta)

    def c(self):
        it = list(self.iters) + [0] * (4 - len(self.iters))
        dm = list(self.d_max) + [self.d_max[-1]] * (4 - len(self.d_max))
        return ups_icp_params(self.levels, (ctypes.c_int32 * 4)(*it), (ctypes.c_float * 4)(*dm),
                              self.cos_theta_max, self.stop_update_norm, self.min_inliers, self.precision,
                              self.irls_delta)


@dataclass
class FuseParams:
    d_max: float = 0.2
    cos_theta_max: float = math.cos(math.radians(30.0))
    min_cos_incidence: float = 0.1
    max_count: int = 10

    def c(self):
        return ups_fuse_params(self.d_max, self.cos_theta_max, self.min_cos_incidence, self.max_count)


def geom_c(g) -> ups_geom:
    """Any object with rows, cols, el_top, d_el, r_min, r_max."""
    return ups_geom(int(g.rows), int(g.cols), float(g.el_top), float(g.d_el), float(g.r_min), float(g.r_max))


# ----------------------------------------------------------------------------
# torch plumbing
# ----------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream():
    return _P(_torch().cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype, what):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise UpsError(f"{what} must be a CUDA tensor")
    if t.dtype != dtype:
        raise UpsError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise UpsError(f"{what} must be contiguous")
    return _P(t.data_ptr())


def pose_tensor(T, device="cuda"):
    """Device FP64 pose (ups_pose layout: R row-major then t) from a 4x4."""
    torch = _torch()
    T = np.asarray(T, dtype=np.float64)
    flat = np.concatenate([T[:3, :3].reshape(9), T[:3, 3]])
    return torch.tensor(flat, dtype=torch.float64, device=device)


def pose_from_tensor(t) -> np.ndarray:
    p = t.detach().cpu().numpy().astype(np.float64)
    T = np.eye(4)
    T[:3, :3] = p[:9].reshape(3, 3)
    T[:3, 3] = p[9:12]
    return T


class Context:
    """A library context: device scratch for panoramas up to ``max_pixels``
    pixels and batches of ``max_batch`` registrations totalling
    ``max_batch_pixels`` pixels."""

    def __init__(self, device: int = 0, max_pixels: int = 1 << 20, max_batch: int = 0, max_batch_pixels: int = 0):
        lib = load()
        h = _P()
        _check(lib.ups_context_create(ctypes.byref(h), int(device), int(max_pixels), int(max_batch),
                                      int(max_batch_pixels)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _LIB.ups_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def new_result(device="cuda"):
    torch = _torch()
    return torch.zeros(RESULT_BYTES, dtype=torch.uint8, device=device)


def read_result(res) -> dict:
    return read_result_bytes(bytes(res.detach().cpu().numpy().tobytes()))


def read_neq(t) -> dict:
    r = ups_normal_eq.from_buffer_copy(bytes(t.detach().cpu().numpy().tobytes()))
    return dict(JtJ=np.array(r.JtJ[:]), Jtr=np.array(r.Jtr[:]), sum_r2=r.sum_r2, inliers=r.inliers, valid=r.valid)


# ----------------------------------------------------------------------------
# entry points (same names as the C ABI without the ups_ prefix)
# ----------------------------------------------------------------------------

def panorama_normals(ctx: Context, geom, depth, surfel=None, params: NormalParams | None = None):
    torch = _torch()
    p = (params or NormalParams()).c()
    if surfel is None:
        surfel = torch.empty((geom.rows, geom.cols, 4), dtype=torch.float32, device=depth.device)
    g = geom_c(geom)
    _check(_LIB.ups_panorama_normals(ctx.handle, ctypes.byref(g), _dev_ptr(depth, torch.float32, "depth"),
                                     _dev_ptr(surfel, torch.float32, "surfel"), ctypes.byref(p), _stream()))
    return surfel


def pyramid_level(ctx: Context, geom, surfel, level: int, out=None):
    torch = _torch()
    if out is None:
        out = torch.empty((geom.rows >> level, geom.cols >> level, 4), dtype=torch.float32, device=surfel.device)
    g = geom_c(geom)
    _check(_LIB.ups_pyramid_level(ctx.handle, ctypes.byref(g), _dev_ptr(surfel, torch.float32, "surfel"),
                                  int(level), _dev_ptr(out, torch.float32, "out"), _stream()))
    return out


def host_pose(T) -> ups_pose:
    """Host ups_pose from a 4x4."""
    T = np.asarray(T, dtype=np.float64)
    p = ups_pose()
    for k in range(9):
        p.R[k] = float(T[k // 3, k % 3])
    for k in range(3):
        p.t[k] = float(T[k, 3])
    return p


def register_scan(ctx: Context, scan_geom, scan_surfel, kf_geom, kf_surfel, init, params: IcpParams | None = None,
                  result=None, world_kf=None):
    """``init``: a 4x4 (host) or a device FP64 pose tensor.  Returns the device
    result buffer (``read_result`` decodes it).  ``world_kf``: a 4x4 keyframe
    world pose selects the world-frame FP32 variant (precision study)."""
    torch = _torch()
    p = (params or IcpParams()).c()
    if result is None:
        result = new_result(scan_surfel.device)
    if isinstance(init, torch.Tensor):
        init_t = init
    else:
        init_t = pose_tensor(init, scan_surfel.device)
    sg, kg = geom_c(scan_geom), geom_c(kf_geom)
    if world_kf is None:
        _check(_LIB.ups_register_scan(ctx.handle, ctypes.byref(sg),
                                      _dev_ptr(scan_surfel, torch.float32, "scan surfel"), ctypes.byref(kg),
                                      _dev_ptr(kf_surfel, torch.float32, "keyframe surfel"),
                                      _dev_ptr(init_t, torch.float64, "init pose"), ctypes.byref(p),
                                      _dev_ptr(result, torch.uint8, "result"), _stream()))
    else:
        w = host_pose(world_kf)
        _check(_LIB.ups_register_scan_world(ctx.handle, ctypes.byref(sg),
                                            _dev_ptr(scan_surfel, torch.float32, "scan surfel"), ctypes.byref(kg),
                                            _dev_ptr(kf_surfel, torch.float32, "keyframe surfel"), ctypes.byref(w),
                                            _dev_ptr(init_t, torch.float64, "init pose"), ctypes.byref(p),
                                            _dev_ptr(result, torch.uint8, "result"), _stream()))
    result._keep_init = init_t  # keep a host-made init alive until the stream consumes it
    return result


def register_scan_noalloc(scan_geom, scan_surfel, kf_geom, kf_surfel, init, params: IcpParams | None = None,
                          result=None):
    """``register_scan`` through the entry point that allocates nothing (its
    scratch is a static device array; panoramas up to 262144 pixels), on the
    current device.  ``init`` and ``result`` as for ``register_scan``."""
    torch = _torch()
    p = (params or IcpParams()).c()
    if result is None:
        result = new_result(scan_surfel.device)
    init_t = init if isinstance(init, torch.Tensor) else pose_tensor(init, scan_surfel.device)
    sg, kg = geom_c(scan_geom), geom_c(kf_geom)
    _check(_LIB.ups_register_scan_noalloc(ctypes.byref(sg), _dev_ptr(scan_surfel, torch.float32, "scan surfel"),
                                          ctypes.byref(kg), _dev_ptr(kf_surfel, torch.float32, "keyframe surfel"),
                                          _dev_ptr(init_t, torch.float64, "init pose"), ctypes.byref(p),
                                          _dev_ptr(result, torch.uint8, "result"), _stream()))
    result._keep_init = init_t
    return result


def result_pose(result):
    """Device view of the pose inside a result buffer (for fuse_scan)."""
    return result[: ctypes.sizeof(ups_pose)].view(_torch().float64)


def fuse_scan(ctx: Context, scan_geom, scan_surfel, kf_geom, kf_surfel, kf_count, T, params: FuseParams | None = None):
    torch = _torch()
    p = (params or FuseParams()).c()
    T_t = T if isinstance(T, torch.Tensor) else pose_tensor(T, scan_surfel.device)
    sg, kg = geom_c(scan_geom), geom_c(kf_geom)
    _check(_LIB.ups_fuse_scan(ctx.handle, ctypes.byref(sg), _dev_ptr(scan_surfel, torch.float32, "scan surfel"),
                              ctypes.byref(kg), _dev_ptr(kf_surfel, torch.float32, "keyframe surfel"),
                              _dev_ptr(kf_count, torch.int16, "keyframe count") if kf_count.dtype == torch.int16
                              else _dev_ptr(kf_count, torch.uint16, "keyframe count"),
                              _dev_ptr(T_t, torch.float64, "pose"), ctypes.byref(p), _stream()))
    return kf_surfel, kf_count


def splat_sweep(ctx: Context, raw_geom, raw, col_T=None, out_geom=None, out=None):
    """Panorama of ``out_geom`` (default: the sweep's own geometry) from a
    sweep's ranges ``raw`` (device float32 [rows, cols]); ``col_T``: per-column
    transforms into the reference frame as a device float32 [cols, 12] tensor,
    a host array [cols, 4, 4] / [cols, 12], or None for the identity."""
    torch = _torch()
    dev = raw.device
    og = out_geom or raw_geom
    if col_T is not None and not isinstance(col_T, torch.Tensor):
        a = np.asarray(col_T, dtype=np.float64)
        if a.ndim == 3:
            a = np.concatenate([a[:, :3, :3].reshape(-1, 9), a[:, :3, 3]], axis=1)
        col_T = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    if out is None:
        out = torch.empty((og.rows, og.cols), dtype=torch.float32, device=dev)
    rg, oc = geom_c(raw_geom), geom_c(og)
    _check(_LIB.ups_splat_sweep(ctx.handle, ctypes.byref(rg), _dev_ptr(raw, torch.float32, "raw ranges"),
                                None if col_T is None else _dev_ptr(col_T, torch.float32, "column transforms"),
                                ctypes.byref(oc), _dev_ptr(out, torch.float32, "depth"), _stream()))
    out._keep = col_T
    return out


class ups_consistency_params(ctypes.Structure):
    _fields_ = [("margin_abs", ctypes.c_float), ("margin_rel", ctypes.c_float), ("min_count", ctypes.c_int32)]


LOOP_NONE, LOOP_WEAK, LOOP_STRONG = 0, 1, 2


@dataclass
class ConsistencyParams:
    """Moving-object check across keyframes: a sample is removed when the other
    keyframe saw more than max(margin_abs, margin_rel * range) beyond it on
    every ray of a 3x3 neighbourhood, each with >= min_count samples."""
    margin_abs: float = 0.2
    margin_rel: float = 0.02
    min_count: int = 1

    def c(self):
        return ups_consistency_params(self.margin_abs, self.margin_rel, self.min_count)


def _count_ptr(t, what):
    torch = _torch()
    if t is None:
        return None
    return _dev_ptr(t, torch.int16 if t.dtype == torch.int16 else torch.uint16, what)


def keyframe_consistency(ctx: Context, a_geom, a_surfel, a_count, b_geom, b_surfel, b_count, T_ba,
                         params: ConsistencyParams | None = None, mutual: bool = True, a_mask=None, b_mask=None,
                         removed=None):
    """Remove in place the samples of keyframe A (and of B when ``mutual``)
    that the other keyframe looked through; counts may be None.  Returns the
    device masks (uint8, 1 = removed; B's is None unless mutual) and the
    device int32 [2] removal counts."""
    torch = _torch()
    dev = a_surfel.device
    p = (params or ConsistencyParams()).c()
    T_t = T_ba if isinstance(T_ba, torch.Tensor) else pose_tensor(T_ba, dev)
    if a_mask is None:
        a_mask = torch.empty((a_geom.rows, a_geom.cols), dtype=torch.uint8, device=dev)
    if mutual and b_mask is None:
        b_mask = torch.empty((b_geom.rows, b_geom.cols), dtype=torch.uint8, device=dev)
    if not mutual:
        b_mask = None
    if removed is None:
        removed = torch.empty(2, dtype=torch.int32, device=dev)
    ga, gb = geom_c(a_geom), geom_c(b_geom)
    _check(_LIB.ups_keyframe_consistency(ctx.handle, ctypes.byref(ga), _dev_ptr(a_surfel, torch.float32, "A surfel"),
                                         _count_ptr(a_count, "A count"), ctypes.byref(gb),
                                         _dev_ptr(b_surfel, torch.float32, "B surfel"), _count_ptr(b_count, "B count"),
                                         _dev_ptr(T_t, torch.float64, "pose"), ctypes.byref(p),
                                         _dev_ptr(a_mask, torch.uint8, "A mask"),
                                         None if b_mask is None else _dev_ptr(b_mask, torch.uint8, "B mask"),
                                         _dev_ptr(removed, torch.int32, "removed"), _stream()))
    a_mask._keep = T_t
    return a_mask, b_mask, removed


def classify_loop_closures(ctx: Context, results, new_keyframe_ratio: float, n: int | None = None):
    """Classes (LOOP_NONE / LOOP_WEAK / LOOP_STRONG, device int32 [n]) of the
    registrations in the device results buffer, and the index of the best
    strong closure (device int32 [1], -1 if none)."""
    torch = _torch()
    n = results.shape[0] if n is None else n
    cls = torch.empty(n, dtype=torch.int32, device=results.device)
    best = torch.empty(1, dtype=torch.int32, device=results.device)
    _check(_LIB.ups_classify_loop_closures(ctx.handle, int(n), _dev_ptr(results, torch.uint8, "results"),
                                           float(new_keyframe_ratio), _dev_ptr(cls, torch.int32, "class"),
                                           _dev_ptr(best, torch.int32, "best"), _stream()))
    return cls, best


def correspondences(ctx: Context, scan_geom, scan_surfel, kf_geom, kf_surfel, T, d_max=0.5,
                    cos_theta_max=math.cos(math.radians(30.0)), world_kf=None):
    """(kf_index, inlier) device maps at the pose T; ``world_kf`` (4x4) selects
    the world-frame FP32 variant."""
    torch = _torch()
    dev = scan_surfel.device
    T_t = T if isinstance(T, torch.Tensor) else pose_tensor(T, dev)
    idx = torch.empty((scan_geom.rows, scan_geom.cols), dtype=torch.int32, device=dev)
    inl = torch.empty((scan_geom.rows, scan_geom.cols), dtype=torch.uint8, device=dev)
    sg, kg = geom_c(scan_geom), geom_c(kf_geom)
    if world_kf is None:
        _check(_LIB.ups_correspondences(ctx.handle, ctypes.byref(sg), _dev_ptr(scan_surfel, torch.float32, "scan"),
                                        ctypes.byref(kg), _dev_ptr(kf_surfel, torch.float32, "keyframe"),
                                        _dev_ptr(T_t, torch.float64, "pose"), float(d_max), float(cos_theta_max),
                                        _dev_ptr(idx, torch.int32, "kf_index"), _dev_ptr(inl, torch.uint8, "inlier"),
                                        _stream()))
    else:
        w = host_pose(world_kf)
        _check(_LIB.ups_correspondences_world(ctx.handle, ctypes.byref(sg),
                                              _dev_ptr(scan_surfel, torch.float32, "scan"), ctypes.byref(kg),
                                              _dev_ptr(kf_surfel, torch.float32, "keyframe"), ctypes.byref(w),
                                              _dev_ptr(T_t, torch.float64, "pose"), float(d_max),
                                              float(cos_theta_max), _dev_ptr(idx, torch.int32, "kf_index"),
                                              _dev_ptr(inl, torch.uint8, "inlier"), _stream()))
    idx._keep = T_t
    return idx, inl


def project_points(ctx: Context, geom, xyz):
    """Nearest pixel (row, col) of each point of a float32 [N, 3] tensor;
    -1 where there is none."""
    torch = _torch()
    n = xyz.shape[0]
    ii = torch.empty(n, dtype=torch.int32, device=xyz.device)
    jj = torch.empty(n, dtype=torch.int32, device=xyz.device)
    g = geom_c(geom)
    _check(_LIB.ups_project_points(ctx.handle, ctypes.byref(g), _dev_ptr(xyz, torch.float32, "points"), int(n),
                                   _dev_ptr(ii, torch.int32, "rows"), _dev_ptr(jj, torch.int32, "cols"), _stream()))
    return ii, jj


def normal_equations(ctx: Context, scan_geom, scan_surfel, kf_geom, kf_surfel, T, d_max=0.5,
                     cos_theta_max=math.cos(math.radians(30.0)), precision=PREC_KAHAN_F64):
    torch = _torch()
    dev = scan_surfel.device
    T_t = T if isinstance(T, torch.Tensor) else pose_tensor(T, dev)
    out = torch.zeros(NEQ_BYTES, dtype=torch.uint8, device=dev)
    sg, kg = geom_c(scan_geom), geom_c(kf_geom)
    _check(_LIB.ups_normal_equations(ctx.handle, ctypes.byref(sg), _dev_ptr(scan_surfel, torch.float32, "scan"),
                                     ctypes.byref(kg), _dev_ptr(kf_surfel, torch.float32, "keyframe"),
                                     _dev_ptr(T_t, torch.float64, "pose"), float(d_max), float(cos_theta_max),
                                     int(precision), _dev_ptr(out, torch.uint8, "out"), _stream()))
    out._keep = T_t
    return out


def debug_reverse_tile_order(reversed_: bool):
    """Debug: later registration launches deal their tiles to workgroups in
    reverse order (results must not change)."""
    _check(_LIB.ups_debug_reverse_tile_order(1 if reversed_ else 0))


def debug_level_spin_limit(polls: int):
    """Debug: a waiting workgroup of a later one-XCD level kernel gives up
    after `polls` unsuccessful polls (0: at its first) and the registration
    ends as DEGENERATE; a negative value restores the default limit."""
    _check(_LIB.ups_debug_level_spin_limit(int(polls)))


# ----------------------------------------------------------------------------
# batches
# ----------------------------------------------------------------------------

def autotune(ctx: Context, cache_path: str | None = None):
    """Measure (or load from ``cache_path``) the pixels per thread of batch
    launches for this GPU."""
    _check(_LIB.ups_autotune(ctx.handle, cache_path.encode() if cache_path else None))


class ups_grid_params(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("n_yaw", ctypes.c_int32), ("n_xy", ctypes.c_int32),
                ("xy_step", ctypes.c_float), ("d_max", ctypes.c_float), ("cos_theta_max", ctypes.c_float)]


@dataclass
class GridParams:
    """Loop-closure grid search: pyramid level scored, yaw samples over the
    turn, translation samples per axis and their spacing (m), Omega
    thresholds of the check.  The default is 36 x 3 x 3 = 324 candidates at
    level 2 with the level-2 registration gate."""
    level: int = 2
    n_yaw: int = 36
    n_xy: int = 3
    xy_step: float = 1.0
    d_max: float = 2.0
    cos_theta_max: float = math.cos(math.radians(30.0))

    def c(self) -> ups_grid_params:
        return ups_grid_params(int(self.level), int(self.n_yaw), int(self.n_xy), float(self.xy_step),
                               float(self.d_max), float(self.cos_theta_max))


class Batch:
    """A planned batch of registrations.  ``items``: dicts with ``scan_geom``,
    ``kf_geom``, device ``scan_surfel`` / ``kf_surfel`` float32 [rows, cols, 4]
    tensors and optional ``scan_depth`` / ``kf_depth`` float32 [rows, cols]
    tensors (for ``normals``).  The tensors must stay alive while the batch
    is used."""

    def __init__(self, ctx: Context, items, params: IcpParams | None = None, pixels_per_thread: int = 0):
        torch = _torch()
        self.ctx = ctx
        self.n = len(items)
        self.items = items
        arr = (ups_batch_item * self.n)()
        for k, it in enumerate(items):
            a = arr[k]
            a.scan_g = geom_c(it["scan_geom"])
            a.kf_g = geom_c(it["kf_geom"])
            a.scan_surfel_d = _dev_ptr(it["scan_surfel"], torch.float32, "scan surfel").value
            a.kf_surfel_d = _dev_ptr(it["kf_surfel"], torch.float32, "keyframe surfel").value
            a.scan_depth_d = _dev_ptr(it["scan_depth"], torch.float32, "scan depth").value \
                if it.get("scan_depth") is not None else None
            a.kf_depth_d = _dev_ptr(it["kf_depth"], torch.float32, "keyframe depth").value \
                if it.get("kf_depth") is not None else None
        self.params = params or IcpParams()
        pc = self.params.c()
        h = _P()
        _check(_LIB.ups_batch_create(ctx.handle, self.n, ctypes.cast(arr, _P), ctypes.byref(pc),
                                     int(pixels_per_thread), ctypes.byref(h)))
        self._h = h

    def fallback(self, results, min_inlier_ratio: float):
        """Rerun from the identity the registrations whose ``results`` (from
        ``register``) have an inlier ratio below ``min_inlier_ratio``; keep
        the better of the two by truncated cost (status FALLBACK_USED)."""
        torch = _torch()
        _check(_LIB.ups_register_batch_fallback(self.ctx.handle, self._h, float(min_inlier_ratio),
                                                _dev_ptr(results, torch.uint8, "results"), _stream()))
        return results

    def fallback_plan(self, results, min_inlier_ratio: float, count=None):
        """First half of ``fallback``: flag the registrations to rerun; their
        number goes to ``count`` (device int32 [1]) if given."""
        torch = _torch()
        cp = None if count is None else _dev_ptr(count, torch.int32, "count")
        _check(_LIB.ups_batch_fallback_plan(self.ctx.handle, self._h, float(min_inlier_ratio),
                                            _dev_ptr(results, torch.uint8, "results"), cp, _stream()))

    def fallback_run(self, results):
        """Second half of ``fallback``: rerun the flagged registrations and merge."""
        torch = _torch()
        _check(_LIB.ups_batch_fallback_run(self.ctx.handle, self._h, _dev_ptr(results, torch.uint8, "results"),
                                           _stream()))
        return results

    def grid_search(self, params: "GridParams | None" = None, base=None, scores=None, best=None, best_score=None):
        """Loop-closure grid search: returns (best poses [n, 12] FP64, best
        scores [n] int32, all scores [n, C] int32) as device tensors."""
        torch = _torch()
        gp = params or GridParams()
        C = gp.n_yaw * gp.n_xy * gp.n_xy
        if base is None:
            base = torch.stack([pose_tensor(np.eye(4)) for _ in range(self.n)])
        if scores is None:
            scores = torch.empty((self.n, C), dtype=torch.int32, device="cuda")
        if best is None:
            best = torch.empty((self.n, 12), dtype=torch.float64, device="cuda")
        if best_score is None:
            best_score = torch.empty(self.n, dtype=torch.int32, device="cuda")
        c = gp.c()
        _check(_LIB.ups_batch_grid_search(self.ctx.handle, self._h, ctypes.byref(c),
                                          _dev_ptr(base, torch.float64, "base poses"),
                                          _dev_ptr(scores, torch.int32, "scores"),
                                          _dev_ptr(best, torch.float64, "best poses"),
                                          _dev_ptr(best_score, torch.int32, "best scores"), _stream()))
        self._grid_keep = base
        return best, best_score, scores

    def set_scheduler(self, persistent):
        """Run later register calls as one launch per iteration (False, the
        default) or as one persistent launch (True)."""
        _check(_LIB.ups_batch_set_scheduler(self._h, 1 if persistent else 0))

    def set_pyramid_mode(self, in_normals):
        """True: the last pass of ``normals`` also writes the pyramid levels of
        the images it computes, and later register and grid-search calls
        build only those of the other images (surfels given as they are);
        False (the default): every register / grid-search call builds them
        all.  The same results either way."""
        _check(_LIB.ups_batch_set_pyramid_mode(self._h, 1 if in_normals else 0))

    def set_iterations(self, iters):
        """Gauss-Newton iterations per level (finest first) of later register
        calls, each at most what the batch was created with; 0 skips a level.
        Fallback calls keep the full schedule."""
        it = list(iters) + [0] * (4 - len(iters))
        arr = (ctypes.c_int32 * 4)(*[int(x) for x in it[:4]])
        _check(_LIB.ups_batch_set_iterations(self._h, ctypes.cast(arr, _P)))

    def schedule(self):
        """(blocks of the persistent launch, pixels per thread of a tile per level)."""
        blocks = ctypes.c_int32()
        kpt = (ctypes.c_int32 * 4)()
        _check(_LIB.ups_batch_schedule(self._h, ctypes.byref(blocks), kpt))
        return blocks.value, list(kpt)

    def pixels_per_thread(self):
        out = (ctypes.c_int32 * 4)()
        _check(_LIB.ups_batch_pixels_per_thread(self._h, out))
        return list(out)

    def normals(self, params: NormalParams | None = None):
        p = (params or NormalParams()).c()
        _check(_LIB.ups_batch_normals(self.ctx.handle, self._h, ctypes.byref(p), _stream()))

    def register(self, init, results=None):
        """``init``: device float64 [n, 12] poses (or a list of 4x4).  Returns
        the device results buffer [n, RESULT_BYTES] (``read_results``)."""
        torch = _torch()
        if not isinstance(init, torch.Tensor):
            init = torch.stack([pose_tensor(T) for T in init])
        if results is None:
            results = torch.zeros((self.n, RESULT_BYTES), dtype=torch.uint8, device=init.device)
        _check(_LIB.ups_register_batch(self.ctx.handle, self._h, _dev_ptr(init, torch.float64, "init poses"),
                                       _dev_ptr(results, torch.uint8, "results"), _stream()))
        results._keep = init
        return results

    def time_iteration(self, level: int = 0, n_launches: int = 20) -> float:
        """Average microseconds of one Gauss-Newton launch at ``level`` over
        all registrations (HIP events on the current stream)."""
        us = ctypes.c_float()
        _check(_LIB.ups_batch_time_iteration(self.ctx.handle, self._h, int(level), int(n_launches), _stream(),
                                             ctypes.byref(us)))
        return us.value

    def close(self):
        if getattr(self, "_h", None):
            _LIB.ups_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def read_results(results) -> list:
    raw = results.detach().cpu().numpy()
    return [read_result_bytes(bytes(raw[k].tobytes())) for k in range(raw.shape[0])]


def read_result_bytes(raw: bytes) -> dict:
    r = ups_icp_result.from_buffer_copy(raw)
    T = np.eye(4)
    T[:3, :3] = np.array(r.T.R[:]).reshape(3, 3)
    T[:3, 3] = np.array(r.T.t[:])
    return dict(T=T, rms=r.rms, trunc_cost=r.trunc_cost, inlier_ratio=r.inlier_ratio, inliers=r.inliers,
                valid=r.valid, iters_run=r.iters_run, status=r.status, level_iters=list(r.level_iters),
                JtJ=np.array(r.JtJ[:]),
                Jtr=np.array(r.Jtr[:]), last_update_norm=r.last_update_norm)


# ---------------------------------------------------------------------------
# learned pose proposal
# ---------------------------------------------------------------------------

PROPOSAL_ROWS, PROPOSAL_COLS = 32, 256


class ups_range_image(ctypes.Structure):
    _fields_ = [("range_d", _P), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32), ("stride", ctypes.c_int32),
                ("r_min", ctypes.c_float), ("r_max", ctypes.c_float)]


def range_image(t, geom=None):
    """Descriptor of a device range source: a float32 depth image [rows, cols]
    or the range channel of a surfel image [rows, cols, 4]."""
    torch = _torch()
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise UpsError("range source must be a contiguous CUDA float32 tensor")
    if t.dim() == 3 and t.shape[2] == 4:
        ptr, stride = t.data_ptr() + 12, 4
    elif t.dim() == 2:
        ptr, stride = t.data_ptr(), 1
    else:
        raise UpsError("range source must be [rows, cols] or [rows, cols, 4]")
    r_min = float(geom.r_min) if geom is not None else 0.0
    r_max = float(geom.r_max) if geom is not None else 50.0
    return ups_range_image(_P(ptr), int(t.shape[0]), int(t.shape[1]), stride, r_min, r_max)


def proposal_num_params() -> int:
    return int(load().ups_proposal_num_params())


class Proposal:
    """The pose-proposal network on the GPU (parameters, Adam state and
    buffers for batches of up to ``max_batch`` pairs)."""

    def __init__(self, ctx: Context, max_batch: int):
        h = _P()
        _check(load().ups_proposal_create(ctx.handle, int(max_batch), ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.max_batch = max_batch
        self.n_params = proposal_num_params()
        self._planned = None

    def set_params(self, params):
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if a.size != self.n_params:
            raise UpsError("parameter count mismatch")
        _check(_LIB.ups_proposal_set_params(self._h, a.ctypes.data_as(_P), int(a.size)))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.n_params, dtype=np.float32)
        _check(_LIB.ups_proposal_get_params(self._h, a.ctypes.data_as(_P), int(a.size)))
        return a

    def save(self, path: str):
        """Write the parameters to ``path`` (the library's parameter file)."""
        _check(_LIB.ups_proposal_save(self._h, os.fsencode(path)))

    def load(self, path: str):
        """Read parameters written by ``save`` (resets the Adam moments)."""
        _check(_LIB.ups_proposal_load(self._h, os.fsencode(path)))

    def get_grads(self) -> np.ndarray:
        a = np.empty(self.n_params, dtype=np.float32)
        _check(_LIB.ups_proposal_get_grads(self._h, a.ctypes.data_as(_P), int(a.size)))
        return a

    def save_checkpoint(self, path: str):
        """Parameters, Adam moments and step count to ``path``."""
        _check(_LIB.ups_proposal_save_checkpoint(self._h, os.fsencode(path)))

    def load_checkpoint(self, path: str):
        """Resume from a file written by ``save_checkpoint``."""
        _check(_LIB.ups_proposal_load_checkpoint(self._h, os.fsencode(path)))

    # NHWC shapes of the five convolution outputs
    ACT_SHAPES = ((16, 128, 32), (8, 64, 64), (4, 32, 96), (2, 16, 128), (2, 16, 128))

    def activations(self, layer: int, n: int):
        """(stored output of convolution layer ``layer`` (1..5) as float64
        values of its bfloat16 bits, its FP32 gradient from the last training
        step), each [n, h, w, c]."""
        shape = (n,) + self.ACT_SHAPES[layer - 1]
        a = np.empty(shape, dtype=np.uint16)
        d = np.empty(shape, dtype=np.float32)
        _check(_LIB.ups_proposal_activations(self._h, int(layer), int(n), a.ctypes.data_as(_P),
                                             d.ctypes.data_as(_P)))
        return (a.astype(np.uint32) << 16).view(np.float32).astype(np.float64), d.astype(np.float64)

    def plan_input(self, kf_sources, scan_sources, kf_geoms=None, scan_geoms=None):
        """Record (keyframe, scan) range sources (tensors, see range_image)."""
        n = len(kf_sources)
        kf = (ups_range_image * n)(*[range_image(t, kf_geoms[k] if kf_geoms else None)
                                     for k, t in enumerate(kf_sources)])
        sc = (ups_range_image * n)(*[range_image(t, scan_geoms[k] if scan_geoms else None)
                                     for k, t in enumerate(scan_sources)])
        _check(_LIB.ups_proposal_plan_input(self._h, n, ctypes.cast(kf, _P), ctypes.cast(sc, _P)))
        self._planned = (n, list(kf_sources), list(scan_sources))

    def input(self, x=None):
        """Network input of the planned pairs into ``x`` (bfloat16 [n, 32, 256, 2])
        or, when None, into the proposal's own buffer."""
        torch = _torch()
        ptr = None if x is None else _dev_ptr(x, torch.bfloat16, "input")
        _check(_LIB.ups_proposal_input(self._h, ptr, _stream()))
        return x

    def forward(self, n: int, x=None, y=None):
        torch = _torch()
        if y is None:
            y = torch.empty((n, 6), dtype=torch.float32, device="cuda")
        ptr = None if x is None else _dev_ptr(x, torch.bfloat16, "input")
        _check(_LIB.ups_proposal_forward(self._h, int(n), ptr, _dev_ptr(y, torch.float32, "output"), _stream()))
        return y

    def poses(self, y, poses=None):
        torch = _torch()
        n = y.shape[0]
        if poses is None:
            poses = torch.empty((n, 12), dtype=torch.float64, device=y.device)
        _check(_LIB.ups_proposal_poses(self._h, int(n), _dev_ptr(y, torch.float32, "output"),
                                       _dev_ptr(poses, torch.float64, "poses"), _stream()))
        return poses

    def train_step(self, x, target, lr: float, loss=None):
        torch = _torch()
        n = target.shape[0]
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device="cuda")
        xp = None if x is None else _dev_ptr(x, torch.bfloat16, "input")
        _check(_LIB.ups_proposal_train_step(self._h, int(n), xp, _dev_ptr(target, torch.float32, "target"),
                                            float(lr), _dev_ptr(loss, torch.float32, "loss"), _stream()))
        return loss

    def close(self):
        if getattr(self, "_h", None):
            _LIB.ups_proposal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def conv3x3_forward(x, w_nk, b, cout, stride):
    """y = relu(conv(x) + b); x bfloat16 [n, h, w, cin], w_nk bfloat16 [cout, 9 cin]."""
    torch = _torch()
    n, h, w, cin = x.shape
    ho, wo = (h - 1) // stride + 1, (w - 1) // stride + 1
    y = torch.empty((n, ho, wo, cout), dtype=torch.bfloat16, device=x.device)
    _check(load().ups_conv3x3_forward(n, h, w, cin, cout, stride, _dev_ptr(x, torch.bfloat16, "x"),
                                      _dev_ptr(w_nk, torch.bfloat16, "w"), _dev_ptr(b, torch.float32, "b"),
                                      _dev_ptr(y, torch.bfloat16, "y"), _stream()))
    return y


def conv3x3_backward_data(y, dy, w_kn, h, w, cin, stride):
    torch = _torch()
    n, _, _, cout = y.shape
    dx = torch.empty((n, h, w, cin), dtype=torch.float32, device=y.device)
    _check(load().ups_conv3x3_backward_data(n, h, w, cin, cout, stride, _dev_ptr(y, torch.bfloat16, "y"),
                                            _dev_ptr(dy, torch.float32, "dy"), _dev_ptr(w_kn, torch.bfloat16, "w"),
                                            _dev_ptr(dx, torch.float32, "dx"), _stream()))
    return dx


def conv3x3_backward_weight(x, y, dy, stride):
    torch = _torch()
    n, h, w, cin = x.shape
    cout = y.shape[3]
    lib = load()
    wf = int(lib.ups_conv3x3_backward_weight_work(n, h, w, cin, cout, stride))
    if wf < 0:
        raise UpsError("invalid convolution shape")
    work = torch.empty(max(wf, 1), dtype=torch.float32, device=x.device)
    dw = torch.empty((9 * cin, cout), dtype=torch.float32, device=x.device)
    db = torch.empty(cout, dtype=torch.float32, device=x.device)
    _check(lib.ups_conv3x3_backward_weight(n, h, w, cin, cout, stride, _dev_ptr(x, torch.bfloat16, "x"),
                                           _dev_ptr(y, torch.bfloat16, "y"), _dev_ptr(dy, torch.float32, "dy"),
                                           _dev_ptr(dw, torch.float32, "dw"), _dev_ptr(db, torch.float32, "db"),
                                           _dev_ptr(work, torch.float32, "work"), wf, _stream()))
    return dw, db
