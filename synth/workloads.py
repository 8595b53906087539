"""Seeded workloads at the shapes of the paper's sensor (a 64-beam spinning
lidar swept at 10 Hz; keyframes of 1024x128 and 2048x256) and of the five
benchmark configurations of this project.

Each function returns plain numpy data: FP32 range images, FP64 ground-truth
poses and the geometry.  Nothing here computes normals, projections or
registrations.
"""
from __future__ import annotations

import math

import numpy as np

from . import Geom, inv, lidar_geom, outdoor_scene, render, render_sweep, room_scene, rot_x, rot_y, rot_z, se3

DEG = math.pi / 180.0


def _unit_horizontal(rng):
    a = rng.uniform(0, 2 * math.pi)
    return np.array([math.cos(a), math.sin(a), 0.0])


# ----------------------------------------------------------------------------
# configuration 0: one 64x512 scan against one 64x512 keyframe in the box room
# ----------------------------------------------------------------------------

def config0(scene_seed: int = 0, noise_seed: int = 1, rows: int = 64, cols: int = 512, noise: float = 0.01,
            with_boxes: bool = True, want_normals: bool = False, dtype=np.float32):
    """Box room 20x10x4 m with 5 boxes; keyframe sensor at (0, 0, 1.5) m; the
    scan is displaced by 2 deg yaw, 1 deg roll and 0.1 m along a seeded
    horizontal direction.  Returns dict(geom, kf, scan, T_gt, T_world_kf, ...)
    where T_gt = T_kf_scan."""
    g = lidar_geom(rows, cols)
    rng = np.random.Generator(np.random.PCG64(scene_seed + 7919))
    d = _unit_horizontal(rng)
    T_w_kf = se3(np.eye(3), [0.0, 0.0, 1.5])
    T_gt = se3(rot_z(2 * DEG) @ rot_x(1 * DEG), 0.1 * d)
    T_w_s = T_w_kf @ T_gt
    scene = room_scene(scene_seed, sensor_positions=[T_w_kf[:3, 3], T_w_s[:3, 3]], with_boxes=with_boxes)
    out = dict(geom=g, T_gt=T_gt, T_world_kf=T_w_kf, T_world_scan=T_w_s, scene=scene)
    if want_normals:
        out["kf"], out["kf_normals"] = render(scene, g, T_w_kf, noise, noise_seed, want_normals=True, dtype=dtype)
        out["scan"], out["scan_normals"] = render(scene, g, T_w_s, noise, noise_seed + 1, want_normals=True,
                                                  dtype=dtype)
    else:
        out["kf"] = render(scene, g, T_w_kf, noise, noise_seed, dtype=dtype)
        out["scan"] = render(scene, g, T_w_s, noise, noise_seed + 1, dtype=dtype)
    return out


# ----------------------------------------------------------------------------
# configuration 1: sensor-scale outdoor sequence
# ----------------------------------------------------------------------------

def _ground_z(scene, xy):
    return float(scene.ground_height(np.asarray(xy, float).reshape(1, 2))[0])


def random_motion(rng, max_angle, max_trans, yaw_frac=0.8, max_z=None):
    """A rigid motion with rotation angle <= max_angle (mostly yaw) and
    translation length <= max_trans."""
    yaw = rng.uniform(-1, 1) * max_angle * yaw_frac
    rem = math.sqrt(max(0.0, max_angle ** 2 - yaw ** 2))
    roll = rng.uniform(-1, 1) * rem / math.sqrt(2)
    pitch = rng.uniform(-1, 1) * rem / math.sqrt(2)
    R = rot_z(yaw) @ rot_y(pitch) @ rot_x(roll)
    t = rng.normal(size=3)
    if max_z is not None:
        t[2] = 0.0
    t = t / np.linalg.norm(t) * rng.uniform(0.2, 1.0) * max_trans
    if max_z is not None:
        t[2] = rng.uniform(-max_z, max_z)
    return se3(R, t)


def config1(seed: int = 11, rows: int = 128, cols: int = 1024, n_kf_scans: int = 10, path_len: float = 5.0,
            noise: float = 0.01, max_angle=5 * DEG, max_trans=0.5, world_offset=(0.0, 0.0), dtype=np.float32):
    """Outdoor scene; ``n_kf_scans`` scans along a ``path_len`` m path whose
    fusion forms the keyframe (in the frame of the first scan); an extra scan
    displaced from the last one by up to ``max_angle`` / ``max_trans``.

    Returns dict(geom, kf_scans [list of ranges], T_kf_scans [list of 4x4],
    scan, T_gt, T_init, T_world_kf, scene)."""
    g = lidar_geom(rows, cols)
    rng = np.random.Generator(np.random.PCG64(seed))
    off = np.array([world_offset[0], world_offset[1]], dtype=np.float64)
    n = n_kf_scans
    xs = np.linspace(0.0, path_len, n)
    ys = 0.3 * np.sin(xs / path_len * math.pi)
    path = np.stack([xs, ys], axis=1) + off
    scene = outdoor_scene(seed + 1, path)
    poses = []
    for k in range(n):
        heading = math.atan2(0.3 * math.pi / path_len * math.cos(xs[k] / path_len * math.pi), 1.0)
        R = rot_z(heading + rng.uniform(-1, 1) * DEG) @ rot_y(rng.uniform(-0.5, 0.5) * DEG) @ rot_x(
            rng.uniform(-0.5, 0.5) * DEG)
        z = 1.8 + _ground_z(scene, path[k])
        poses.append(se3(R, [path[k, 0], path[k, 1], z]))
    delta = random_motion(rng, rng.uniform(0.5, 1.0) * max_angle, max_trans, max_z=0.05)
    T_w_last = poses[-1] @ delta
    T_w_kf = poses[0]
    scans = [render(scene, g, P, noise, seed * 1000 + k, dtype=dtype) for k, P in enumerate(poses)]
    scan = render(scene, g, T_w_last, noise, seed * 1000 + n, dtype=dtype)
    T_kf_scans = [inv(T_w_kf) @ P for P in poses]
    return dict(geom=g, kf_scans=scans, T_kf_scans=T_kf_scans, scan=scan, T_gt=inv(T_w_kf) @ T_w_last,
                T_init=T_kf_scans[-1], T_world_kf=T_w_kf, T_world_scan=T_w_last, scene=scene)


# ----------------------------------------------------------------------------
# configuration 2: many independent registrations of uneven sizes
# ----------------------------------------------------------------------------

BATCH_SIZES = ((64, 512), (64, 1024), (128, 1024), (128, 2048))


def batch_pair(k: int, base_seed: int = 1000, max_angle=10 * DEG, max_trans=1.0, sizes=BATCH_SIZES,
               noise: float = 0.01, dtype=np.float32, size=None):
    """Registration pair k: scene kind by a seeded coin, panorama size uniform
    over ``sizes``, motion with yaw up to the limit, roll/pitch up to 3 deg,
    translation in a ``max_trans`` ball with |z| <= 0.2 m."""
    seed = base_seed + k
    rng = np.random.Generator(np.random.PCG64(seed))
    rows, cols = sizes[int(rng.integers(len(sizes)))] if size is None else size
    g = lidar_geom(rows, cols)
    outdoor = bool(rng.integers(2))
    yaw = rng.uniform(-1, 1) * max_angle
    roll = rng.uniform(-3, 3) * DEG
    pitch = rng.uniform(-3, 3) * DEG
    ang = math.sqrt(yaw * yaw + roll * roll + pitch * pitch)
    if ang > max_angle:
        s = max_angle / ang
        yaw, roll, pitch = yaw * s, roll * s, pitch * s
    t = rng.normal(size=3)
    t[2] = 0.0
    t = t / (np.linalg.norm(t) + 1e-12) * max_trans * rng.uniform(0, 1) ** (1 / 3)
    t[2] = rng.uniform(-0.2, 0.2)
    delta = se3(rot_z(yaw) @ rot_y(pitch) @ rot_x(roll), t)
    if outdoor:
        kf_xy = np.array([0.0, 0.0])
        scene = outdoor_scene(seed * 7 + 3, np.stack([kf_xy, kf_xy + t[:2]]))
        z = 1.8 + float(scene.ground_height(kf_xy.reshape(1, 2))[0])
        T_w_kf = se3(rot_z(rng.uniform(0, 2 * math.pi)), [kf_xy[0], kf_xy[1], z])
    else:
        c = np.array([rng.uniform(-3, 3), rng.uniform(-1.5, 1.5), 1.5])
        T_w_kf = se3(rot_z(rng.uniform(-0.5, 0.5)), c)
        T_w_s0 = T_w_kf @ delta
        scene = room_scene(seed * 7 + 3, sensor_positions=[T_w_kf[:3, 3], T_w_s0[:3, 3]])
    T_w_s = T_w_kf @ delta
    kf = render(scene, g, T_w_kf, noise, seed * 2, dtype=dtype)
    scan = render(scene, g, T_w_s, noise, seed * 2 + 1, dtype=dtype)
    return dict(geom=g, kf=kf, scan=scan, T_gt=delta, kind=scene.kind, seed=seed)


def batch(n: int = 256, base_seed: int = 1000, **kw):
    return [batch_pair(k, base_seed, **kw) for k in range(n)]


# ----------------------------------------------------------------------------
# configuration 3: the outdoor sequence far from the world origin
# ----------------------------------------------------------------------------

def world_offset(seed: int, radius: float = 4400.0, at_rim: bool = False):
    """A horizontal offset drawn uniformly in a disk of ``radius`` m (on its
    rim when ``at_rim``), seeded."""
    rng = np.random.Generator(np.random.PCG64(seed + 4409))
    a = rng.uniform(0, 2 * math.pi)
    r = radius if at_rim else radius * math.sqrt(rng.uniform())
    return (r * math.cos(a), r * math.sin(a))


def config3(seed: int = 11, offset=(0.0, 0.0), rows: int = 128, cols: int = 2048, **kw):
    """Configuration 1 at 128x2048, with the whole scene, path and keyframe
    placed at a horizontal world offset (metres).  Ray casting and poses are
    FP64, so the rendered ranges do not depend on the offset beyond FP64
    rounding; T_world_kf carries it."""
    return config1(seed=seed, rows=rows, cols=cols, world_offset=offset, **kw)


# ----------------------------------------------------------------------------
# outlier patches: rectangles of a depth image moved along their rays
# ----------------------------------------------------------------------------

def outlier_patches(depth, seed: int, frac: float = 0.2, h: int = 8, w: int = 16, amp=(0.1, 0.3)):
    """Copy of ``depth`` with about ``frac`` of its pixels in h x w rectangles
    (seeded positions, overlaps allowed) whose returns are moved by one common
    offset per rectangle, |offset| uniform in ``amp`` metres with a random
    sign: surfaces that do not belong to the keyframe's scene (objects that
    moved between the sweeps) but still pass a 0.5 m association gate."""
    rng = np.random.Generator(np.random.PCG64(seed + 104729))
    d = np.array(depth, copy=True)
    rows, cols = d.shape
    for _ in range(int(frac * rows * cols / (h * w))):
        i = int(rng.integers(0, rows - h))
        j = int(rng.integers(0, cols - w))
        off = rng.uniform(*amp) * (1.0 if rng.random() < 0.5 else -1.0)
        blk = d[i:i + h, j:j + w]
        d[i:i + h, j:j + w] = np.where(blk > 0, blk + off, blk)
    return d


# ----------------------------------------------------------------------------
# two keyframes of one room with objects that moved between them
# ----------------------------------------------------------------------------

MOVER_SIZE = (0.6, 0.6, 1.8)  # a person-sized box, metres


def _movers(rng, n, room, avoid, min_dist=1.5):
    out = []
    sx, sy, sz = MOVER_SIZE
    tries = 0
    while len(out) < n and tries < 10000:
        tries += 1
        cx = rng.uniform(room[0] + sx, room[3] - sx)
        cy = rng.uniform(room[1] + sy, room[4] - sy)
        b = np.array([cx - sx / 2, cy - sy / 2, 0.0, cx + sx / 2, cy + sy / 2, sz])
        lo, hi = b[:3], b[3:]
        if any(np.linalg.norm(np.maximum(np.maximum(lo - p, 0), p - hi)) < min_dist for p in avoid):
            continue
        out.append(b)
    return np.array(out).reshape(-1, 6)


def moving_objects_pair(seed: int, rows: int = 64, cols: int = 1024, n_movers: int = 3, baseline: float = 3.0,
                        noise: float = 0.01, dtype=np.float32):
    """Two keyframes of the box room ``baseline`` metres apart.  Person-sized
    boxes stand in the room only when keyframe A is taken (``n_movers`` of
    them) and others only when B is taken.  Returns dict(geom, kf_a, kf_b,
    T_ba (A frame -> B frame), T_world_a, T_world_b, mover_a, mover_b) where
    mover_* marks the pixels whose return comes from a mover (noise-free
    renders with and without the movers differ)."""
    rng = np.random.Generator(np.random.PCG64(seed + 3571))
    pa = np.array([rng.uniform(-5, 5), rng.uniform(-2, 2), 1.5])
    d = _unit_horizontal(rng) * baseline
    pb = pa + np.array([d[0], d[1], 0.0])
    pb[0] = float(np.clip(pb[0], -8.0, 8.0))
    pb[1] = float(np.clip(pb[1], -3.5, 3.5))
    T_w_a = se3(rot_z(rng.uniform(-math.pi, math.pi)), pa)
    T_w_b = se3(rot_z(rng.uniform(-math.pi, math.pi)), pb)
    static = room_scene(seed, sensor_positions=[pa, pb], n_boxes=3)
    room = static.room
    mov_a = _movers(rng, n_movers, room, [pa, pb])
    mov_b = _movers(rng, n_movers, room, [pa, pb])
    g = lidar_geom(rows, cols)
    scene_a = type(static)(room=room, boxes=np.vstack([static.boxes, mov_a]), kind="room")
    scene_b = type(static)(room=room, boxes=np.vstack([static.boxes, mov_b]), kind="room")
    kf_a = render(scene_a, g, T_w_a, noise, seed * 2 + 11, dtype=dtype)
    kf_b = render(scene_b, g, T_w_b, noise, seed * 2 + 12, dtype=dtype)
    mover_a = np.abs(render(scene_a, g, T_w_a, dtype=np.float64) - render(static, g, T_w_a, dtype=np.float64)) > 1e-9
    mover_b = np.abs(render(scene_b, g, T_w_b, dtype=np.float64) - render(static, g, T_w_b, dtype=np.float64)) > 1e-9
    return dict(geom=g, kf_a=kf_a, kf_b=kf_b, T_ba=inv(T_w_b) @ T_w_a, T_world_a=T_w_a, T_world_b=T_w_b,
                mover_a=mover_a, mover_b=mover_b, static=static, movers_a=mov_a, movers_b=mov_b)


# ----------------------------------------------------------------------------
# a closed loop through the outdoor scene (keyframe switching, loop closure)
# ----------------------------------------------------------------------------

def loop_sequence(seed: int = 5, n_scans: int = 64, radius: float = 10.0, rows: int = 64, cols: int = 1024,
                  noise: float = 0.01, laps: float = 1.25, dtype=np.float32):
    """``n_scans`` sweeps along a circle of ``radius`` metres through the
    outdoor scene, ``laps`` times around (past the start again), heading along
    the path with small seeded roll and pitch.  Returns dict(geom, scans
    [list of ranges], T_world [list of 4x4], scene)."""
    g = lidar_geom(rows, cols)
    rng = np.random.Generator(np.random.PCG64(seed + 7877))
    ang = np.linspace(0.0, 2 * math.pi * laps, n_scans)
    path = np.stack([radius * np.cos(ang), radius * np.sin(ang)], axis=1)
    ring = np.stack([radius * np.cos(np.linspace(0, 2 * math.pi, 73)),
                     radius * np.sin(np.linspace(0, 2 * math.pi, 73))], axis=1)
    scene = outdoor_scene(seed + 1, ring)
    poses = []
    for k in range(n_scans):
        heading = ang[k] + math.pi / 2
        R = rot_z(heading) @ rot_y(rng.uniform(-0.5, 0.5) * DEG) @ rot_x(rng.uniform(-0.5, 0.5) * DEG)
        z = 1.8 + _ground_z(scene, path[k])
        poses.append(se3(R, [path[k, 0], path[k, 1], z]))
    scans = [render(scene, g, P, noise, seed * 1000 + k, dtype=dtype) for k, P in enumerate(poses)]
    return dict(geom=g, scans=scans, T_world=poses, scene=scene)


# ----------------------------------------------------------------------------
# a sweep taken while the sensor moves (panorama formation, de-skew)
# ----------------------------------------------------------------------------

def _twist_exp(xi):
    import scipy.linalg
    M = np.zeros((4, 4))
    w, v = xi[:3], xi[3:]
    M[:3, :3] = [[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]
    M[:3, 3] = v
    return scipy.linalg.expm(M)


def moving_sweep(seed: int = 3, rows: int = 64, cols: int = 1024, omega=(0.0, 0.0, math.radians(90.0)),
                 velocity=(0.0, 0.0, 0.0), period: float = 0.1, t_ref: float = 1.0, noise: float = 0.0,
                 outdoor: bool = False, dtype=np.float32):
    """One sweep of ``period`` seconds whose column j fires at time
    t_j = j / cols (fraction of the period) while the sensor turns at the body
    rate ``omega`` (rad/s) and moves at ``velocity`` (m/s, body frame), both
    constant.  The reference instant is t_ref (1: the end of the sweep).
    Returns dict(geom, raw (the sweep as measured), ref (the panorama rendered
    at the reference pose), col_T [cols, 4, 4] (column j's frame -> the
    reference frame: Exp((t_j - t_ref) period xi)), T_world_ref, scene)."""
    g = lidar_geom(rows, cols)
    rng = np.random.Generator(np.random.PCG64(seed + 6151))
    xi = np.concatenate([np.asarray(omega, float), np.asarray(velocity, float)])
    if outdoor:
        p = np.array([0.0, 0.0])
        scene = outdoor_scene(seed + 1, np.stack([p, p + 1.0]))
        T_ref = se3(rot_z(rng.uniform(-math.pi, math.pi)), [0.0, 0.0, 1.8 + float(scene.ground_height(p[None])[0])])
    else:
        pos = np.array([rng.uniform(-3, 3), rng.uniform(-1.5, 1.5), 1.5])
        scene = room_scene(seed, sensor_positions=[pos])
        T_ref = se3(rot_z(rng.uniform(-math.pi, math.pi)), pos)
    col_T = np.stack([_twist_exp((j / cols - t_ref) * period * xi) for j in range(cols)])
    raw = render_sweep(scene, g, T_ref[None] @ col_T, noise, seed * 2 + 1, dtype=dtype)
    ref = render(scene, g, T_ref, noise, seed * 2 + 2, dtype=dtype)
    return dict(geom=g, raw=raw, ref=ref, col_T=col_T, T_world_ref=T_ref, scene=scene, xi=xi, period=period,
                t_ref=t_ref)
