"""Seeded synthetic lidar workloads (input generation only).

This package builds the inputs that both the CPU oracle and the GPU path
consume: panoramic range images rendered by an FP64 ray caster
(``render.c``) from analytic scenes, plus the ground-truth sensor poses.  It
holds none of the registration method's arithmetic (no normals, no
projection of points into panoramas, no association, no solve): it only
draws scene parameters and noise from numpy PCG64 generators and casts rays.

Conventions shared with the method (stated by the paper's problem, not code):

* A panorama has ``rows`` elevation rows and ``cols`` azimuth columns.  Row
  ``i`` looks along elevation ``el_top - i*d_el`` and column ``j`` along
  azimuth ``2*pi*j/cols`` (column 0 along +x, counter-clockwise about +z).
* A pixel stores the Euclidean range to the first surface; 0 means no return.
* Poses are 4x4 homogeneous matrices.  ``T_ab`` maps frame-b coordinates into
  frame a.  The registration target is ``T_kf_scan`` (scan -> keyframe).
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


# ray-casting threads per render when the caller gives none (None: up to 16);
# worker processes that render in parallel set it to 1
DEFAULT_THREADS = None


def _sanitized() -> bool:
    # UPS_SANITIZE=1: a build instrumented with AddressSanitizer and UBSan
    # (clang; its runtime preloaded into the process)
    return os.environ.get("UPS_SANITIZE") == "1"


def _so_path(sanitize):
    return os.path.join(_HERE, "libsynth_san.so" if sanitize else "libsynth.so")


def _lib():
    global _LIB
    if _LIB is None:
        so = _so_path(_sanitized())
        src = os.path.join(_HERE, "render.c")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            build()
        _LIB = ctypes.CDLL(so)
        _LIB.syn_render.restype = ctypes.c_int
    return _LIB


def build(sanitize=None) -> str:
    """Compile the ray caster with gcc (plain C, no fast-math), or with clang
    and the sanitizers."""
    sanitize = _sanitized() if sanitize is None else sanitize
    so = _so_path(sanitize)
    tmp = so + ".tmp%d" % os.getpid()
    if sanitize:
        cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-shared-libsan"]
    else:
        cmd = ["gcc", "-O2"]
    subprocess.check_call(cmd + ["-fno-fast-math", "-fPIC", "-shared", "-o", tmp, os.path.join(_HERE, "render.c"),
                                 "-lm", "-lpthread"])
    os.replace(tmp, so)
    return so


# ----------------------------------------------------------------------------
# sensor geometry
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Geom:
    """Panorama geometry: rows x cols, first-row elevation and row spacing
    (radians), and the valid range interval (r_min, r_max]."""
    rows: int
    cols: int
    el_top: float
    d_el: float
    r_min: float = 0.0
    r_max: float = 50.0

    @property
    def shape(self):
        return (self.rows, self.cols)

    def level(self, l: int) -> "Geom":
        """Geometry of pyramid level l (every 2^l-th row and column)."""
        s = 1 << l
        return Geom(self.rows // s, self.cols // s, self.el_top, self.d_el * s, self.r_min, self.r_max)


def lidar_geom(rows: int, cols: int, r_max: float = 50.0) -> Geom:
    """Endpoint-inclusive beam elevations: 64 rows span +-16.6 deg, 128 rows
    span +-22.5 deg, 32 rows (a downsampled input) span +-22.5 deg."""
    half = {64: 16.6, 128: 22.5}.get(rows, 22.5)
    el_top = math.radians(half)
    d_el = math.radians(2 * half) / (rows - 1)
    return Geom(rows, cols, el_top, d_el, 0.0, r_max)


# ----------------------------------------------------------------------------
# poses
# ----------------------------------------------------------------------------

def rot_x(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]], dtype=np.float64)


def rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]], dtype=np.float64)


def rot_z(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]], dtype=np.float64)


def se3(R=None, t=None):
    T = np.eye(4)
    if R is not None:
        T[:3, :3] = R
    if t is not None:
        T[:3, 3] = t
    return T


def inv(T):
    R, t = T[:3, :3], T[:3, 3]
    return se3(R.T, -R.T @ t)


def rot_angle(R):
    """Geodesic angle of a rotation matrix, stable near 0."""
    d = np.linalg.norm(R - np.eye(3))
    return 2.0 * math.asin(min(1.0, d / (2.0 * math.sqrt(2.0))))


def pose_error(Ta, Tb):
    """(rotation angle in rad, translation distance in m) between two poses,
    computed as 2*asin(|Ra - Rb|_F / (2*sqrt 2)) and |ta - tb|."""
    d = np.linalg.norm(Ta[:3, :3] - Tb[:3, :3])
    rot = 2.0 * math.asin(min(1.0, d / (2.0 * math.sqrt(2.0))))
    return rot, float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3]))


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------

class _SceneC(ctypes.Structure):
    _fields_ = [("has_room", ctypes.c_int), ("room", ctypes.c_double * 6),
                ("nbox", ctypes.c_int), ("boxes", ctypes.c_void_p),
                ("ncyl", ctypes.c_int), ("cyl", ctypes.c_void_p),
                ("nfac", ctypes.c_int), ("fac", ctypes.c_void_p),
                ("has_ground", ctypes.c_int), ("g_amp", ctypes.c_double),
                ("g_scale", ctypes.c_double), ("perm", ctypes.c_void_p)]


class _GeomC(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int), ("cols", ctypes.c_int), ("el_top", ctypes.c_double),
                ("d_el", ctypes.c_double), ("r_max", ctypes.c_double)]


@dataclass
class Scene:
    room: np.ndarray | None = None                       # (6,) min xyz, max xyz
    boxes: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))
    cylinders: np.ndarray = field(default_factory=lambda: np.zeros((0, 5)))
    facades: np.ndarray = field(default_factory=lambda: np.zeros((0, 6)))
    ground_perm: np.ndarray | None = None                # (512,) int32
    ground_amp: float = 0.0
    ground_scale: float = 1.0
    kind: str = ""

    def _c(self):
        keep = []

        def arr(a, cols):
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1, cols))
            keep.append(a)
            return a.shape[0], (a.ctypes.data if a.size else None)

        sc = _SceneC()
        if self.room is not None:
            sc.has_room = 1
            for k in range(6):
                sc.room[k] = float(self.room[k])
        sc.nbox, sc.boxes = arr(self.boxes, 6)
        sc.ncyl, sc.cyl = arr(self.cylinders, 5)
        sc.nfac, sc.fac = arr(self.facades, 6)
        if self.ground_perm is not None:
            p = np.ascontiguousarray(self.ground_perm, dtype=np.int32)
            keep.append(p)
            sc.has_ground = 1
            sc.g_amp = self.ground_amp
            sc.g_scale = self.ground_scale
            sc.perm = p.ctypes.data
        return sc, keep

    def ground_height(self, xy):
        """Height of the ground under world points xy [..., 2] (0 if flat)."""
        xy = np.ascontiguousarray(np.asarray(xy, dtype=np.float64).reshape(-1, 2))
        z = np.zeros(xy.shape[0])
        if self.ground_perm is not None:
            p = np.ascontiguousarray(self.ground_perm, dtype=np.int32)
            _lib().syn_ground_height(p.ctypes.data_as(ctypes.c_void_p), ctypes.c_double(self.ground_amp),
                                     ctypes.c_double(self.ground_scale), ctypes.c_int(xy.shape[0]),
                                     xy.ctypes.data_as(ctypes.c_void_p), z.ctypes.data_as(ctypes.c_void_p))
        return z


def _box_point_dist(box, p):
    lo, hi = box[:3], box[3:]
    d = np.maximum(np.maximum(lo - p, 0), p - hi)
    return float(np.linalg.norm(d))


def room_scene(seed: int, sensor_positions=(), n_boxes: int = 5, with_boxes: bool = True) -> Scene:
    """The 20 x 10 x 4 m box room with ``n_boxes`` axis-aligned boxes (sides
    U[0.5, 2] m) resting on the floor, none within 1 m of any sensor position."""
    rng = np.random.Generator(np.random.PCG64(seed))
    room = np.array([-10.0, -5.0, 0.0, 10.0, 5.0, 4.0])
    boxes = []
    tries = 0
    while with_boxes and len(boxes) < n_boxes and tries < 10000:
        tries += 1
        sx, sy, sz = rng.uniform(0.5, 2.0, size=3)
        cx = rng.uniform(-10 + sx / 2, 10 - sx / 2)
        cy = rng.uniform(-5 + sy / 2, 5 - sy / 2)
        b = np.array([cx - sx / 2, cy - sy / 2, 0.0, cx + sx / 2, cy + sy / 2, sz])
        if any(_box_point_dist(b, np.asarray(p, float)) < 1.0 for p in sensor_positions):
            continue
        boxes.append(b)
    return Scene(room=room, boxes=np.array(boxes).reshape(-1, 6), kind="room")


def outdoor_scene(seed: int, path_xy, n_cyl: int = 200, extent: float = 100.0) -> Scene:
    """Outdoor scene: ground z = 0.05 * noise(x/2, y/2), ``n_cyl`` vertical
    cylinders (r in U[0.1, 0.5] m, heights U[2, 8] m) in an extent x extent
    square avoiding 2 m around the path, and 4 facades 10 m tall placed
    15-30 m from the path."""
    rng = np.random.Generator(np.random.PCG64(seed))
    path_xy = np.asarray(path_xy, dtype=np.float64).reshape(-1, 2)
    center = path_xy.mean(axis=0)
    perm = rng.permutation(256).astype(np.int32)
    perm = np.concatenate([perm, perm])

    def path_dist(p):
        # distance from p to the polyline through path_xy
        best = np.inf
        pts = path_xy if len(path_xy) > 1 else np.vstack([path_xy, path_xy])
        for a, b in zip(pts[:-1], pts[1:]):
            ab = b - a
            L = float(ab @ ab)
            s = 0.0 if L == 0 else float(np.clip((p - a) @ ab / L, 0, 1))
            best = min(best, float(np.linalg.norm(p - (a + s * ab))))
        return best

    cyl = []
    while len(cyl) < n_cyl:
        c = center + rng.uniform(-extent / 2, extent / 2, size=2)
        r = rng.uniform(0.1, 0.5)
        h = rng.uniform(2.0, 8.0)
        if path_dist(c) < 2.0 + r:
            continue
        cyl.append([c[0], c[1], r, -1.0, h])
    fac = []
    for k in range(4):
        ang = k * math.pi / 2 + rng.uniform(-0.3, 0.3)
        dist = rng.uniform(15.0, 30.0)
        length = rng.uniform(15.0, 40.0)
        nrm = np.array([math.cos(ang), math.sin(ang)])
        tan = np.array([-nrm[1], nrm[0]])
        mid = center + dist * nrm + rng.uniform(-5, 5) * tan
        p0, p1 = mid - tan * length / 2, mid + tan * length / 2
        fac.append([p0[0], p0[1], p1[0], p1[1], -1.0, 10.0])
    return Scene(cylinders=np.array(cyl), facades=np.array(fac), ground_perm=perm,
                 ground_amp=0.05, ground_scale=2.0, kind="outdoor")


def render(scene: Scene, geom: Geom, T_world_sensor, noise_sigma: float = 0.0, noise_seed: int | None = None,
           want_normals: bool = False, dtype=np.float32, threads: int | None = None):
    """Ray-cast one panorama from the sensor pose ``T_world_sensor``.

    Returns the range image (``dtype``, 0 = no return).  With ``noise_sigma`` > 0
    Gaussian range noise N(0, sigma) drawn from PCG64(noise_seed) is added to
    valid pixels; pixels pushed outside (r_min, r_max] become 0.  With
    ``want_normals`` the exact sensor-frame surface normals [rows, cols, 3]
    (FP64, facing the sensor) are returned as a second value.
    """
    T = np.asarray(T_world_sensor, dtype=np.float64)
    R = np.ascontiguousarray(T[:3, :3])
    o = np.ascontiguousarray(T[:3, 3])
    rng_ = np.zeros((geom.rows, geom.cols), dtype=np.float64)
    nrm = np.zeros((geom.rows, geom.cols, 3), dtype=np.float64) if want_normals else None
    sc, keep = scene._c()
    g = _GeomC(geom.rows, geom.cols, geom.el_top, geom.d_el, geom.r_max)
    if threads is None:
        threads = DEFAULT_THREADS or min(16, os.cpu_count() or 1)
    _lib().syn_render(ctypes.byref(sc), ctypes.byref(g), R.ctypes.data_as(ctypes.c_void_p),
                      o.ctypes.data_as(ctypes.c_void_p), rng_.ctypes.data_as(ctypes.c_void_p),
                      nrm.ctypes.data_as(ctypes.c_void_p) if nrm is not None else None, None,
                      ctypes.c_int(threads))
    del keep
    if noise_sigma > 0:
        rng = np.random.Generator(np.random.PCG64(noise_seed if noise_seed is not None else 0))
        noise = rng.normal(0.0, noise_sigma, size=rng_.shape)
        valid = rng_ > 0
        rng_ = np.where(valid, rng_ + noise, 0.0)
        rng_ = np.where((rng_ > geom.r_min) & (rng_ <= geom.r_max), rng_, 0.0)
    out = rng_.astype(dtype)
    if want_normals:
        if nrm is not None:
            nrm[out == 0] = 0.0
        return out, nrm
    return out


def render_sweep(scene: Scene, geom: Geom, T_world_cols, noise_sigma: float = 0.0, noise_seed: int | None = None,
                 dtype=np.float32, threads: int | None = None):
    """Ray-cast a sweep taken while the sensor moves: column j (azimuth
    2 pi j / cols, every row) is captured from its own pose T_world_cols[j]
    (array [cols, 4, 4]).  Range image as ``render`` returns it."""
    T = np.asarray(T_world_cols, dtype=np.float64).reshape(geom.cols, 4, 4)
    R = np.ascontiguousarray(T[:, :3, :3].reshape(geom.cols, 9))
    o = np.ascontiguousarray(T[:, :3, 3])
    rng_ = np.zeros((geom.rows, geom.cols), dtype=np.float64)
    sc, keep = scene._c()
    g = _GeomC(geom.rows, geom.cols, geom.el_top, geom.d_el, geom.r_max)
    if threads is None:
        threads = DEFAULT_THREADS or min(16, os.cpu_count() or 1)
    _lib().syn_render_sweep(ctypes.byref(sc), ctypes.byref(g), R.ctypes.data_as(ctypes.c_void_p),
                            o.ctypes.data_as(ctypes.c_void_p), rng_.ctypes.data_as(ctypes.c_void_p),
                            ctypes.c_int(threads))
    del keep
    if noise_sigma > 0:
        rng = np.random.Generator(np.random.PCG64(noise_seed if noise_seed is not None else 0))
        noise = rng.normal(0.0, noise_sigma, size=rng_.shape)
        valid = rng_ > 0
        rng_ = np.where(valid, rng_ + noise, 0.0)
        rng_ = np.where((rng_ > geom.r_min) & (rng_ <= geom.r_max), rng_, 0.0)
    return rng_.astype(dtype)
