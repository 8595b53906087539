"""Keyframe management around the registration path (UPSLAM Section III-C).

Each sweep is registered to the current keyframe and fused into it while the
registration quality -- the inlier ratio -- stays at or above the
new-keyframe threshold.  Below it a new keyframe is sought: the keyframes
near the current pose estimate are loop-closure candidates, each scored by
the grid search over candidate transforms and registered from the best one
(one batched call for all candidates); a strong closure (ratio above the
threshold) makes that keyframe the current one, weak closures (above 3/4 of
it) only add pose-graph edges.  Without a strong closure the sweep itself
becomes a new keyframe.  Whenever the current keyframe changes, the old and
the new keyframe are checked against each other and the samples of moving
objects removed.

The decisions live here, in host code; every step on the data runs in the
library's kernels (``GpuBackend``).  The pose graph is recorded as a list of
edges; its optimisation is not part of this package.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

EDGE_ODOMETRY, EDGE_STRONG, EDGE_WEAK = "odometry", "strong", "weak"
MOTION_ZERO_VELOCITY, MOTION_ZERO_ACCELERATION = "zero_velocity", "zero_acceleration"


def rigid_inv(T):
    T = np.asarray(T, dtype=np.float64)
    o = np.eye(4)
    o[:3, :3] = T[:3, :3].T
    o[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return o


@dataclass
class MapParams:
    """new_keyframe_ratio: the quality threshold (the paper tunes it per
    experiment); search_radius / max_candidates: which keyframes near the
    pose estimate are tried as loop closures; grid: the grid search before a
    loop-closure registration (None: register from the estimate);
    motion_prior: the initial guess of the next sweep, the last pose (zero
    velocity) or its extrapolation by the last motion (zero acceleration)."""
    new_keyframe_ratio: float = 0.7
    search_radius: float = 6.0
    max_candidates: int = 8
    min_loop_gap: int = 1
    motion_prior: str = MOTION_ZERO_VELOCITY
    icp: object = None
    grid: object = "default"
    fuse: object = None
    consistency: object = None


@dataclass
class Keyframe:
    id: int
    T_world: np.ndarray
    data: object = None  # backend-owned images (surfels, counts)


@dataclass
class Edge:
    a: int
    b: int
    T_ab: np.ndarray  # keyframe b's frame -> keyframe a's frame
    kind: str
    ratio: float


@dataclass
class Step:
    """What one sweep did: event is 'fused', 'new_keyframe' or 'switched'."""
    event: str
    keyframe: int
    T_kf: np.ndarray
    T_world: np.ndarray
    ratio: float
    closures: list = field(default_factory=list)  # (keyframe id, class, ratio)
    removed: tuple = (0, 0)


class KeyframeMap:
    def __init__(self, backend, params: MapParams | None = None):
        self.b = backend
        self.p = params or MapParams()
        self.keyframes: list[Keyframe] = []
        self.edges: list[Edge] = []
        self.current = -1
        self._T_last = None   # last sweep's pose in the current keyframe
        self._T_prev = None   # the one before (same keyframe), for the zero-acceleration prior

    # ---- the initial guess of the next sweep in the current keyframe
    def _prior(self):
        if self._T_last is None:
            return np.eye(4)
        if self.p.motion_prior == MOTION_ZERO_ACCELERATION and self._T_prev is not None:
            return self._T_last @ (rigid_inv(self._T_prev) @ self._T_last)
        return self._T_last

    def _set_last(self, T, same_keyframe):
        self._T_prev = self._T_last if same_keyframe else None
        self._T_last = T

    def add_sweep(self, depth) -> Step:
        scan = self.b.normals(depth)
        if self.current < 0:
            kf = Keyframe(0, np.eye(4), self.b.new_keyframe(scan))
            self.keyframes.append(kf)
            self.current = 0
            self._set_last(np.eye(4), False)
            return Step("new_keyframe", 0, np.eye(4), np.eye(4), 1.0)
        cur = self.keyframes[self.current]
        res = self.b.register(scan, cur.data, self._prior())
        T, ratio = res["T"], res["inlier_ratio"]
        ok = res["status"] in (0, 1, 4)
        if ok and ratio >= self.p.new_keyframe_ratio:
            self.b.fuse(scan, cur.data, T)
            self._set_last(T, True)
            return Step("fused", cur.id, T, cur.T_world @ T, ratio)
        # ---- seek a new keyframe: loop closures near the pose estimate
        T_world = cur.T_world @ T
        cands = [k for k in self.keyframes
                 if k.id != cur.id and abs(k.id - cur.id) >= self.p.min_loop_gap
                 and np.linalg.norm(k.T_world[:3, 3] - T_world[:3, 3]) <= self.p.search_radius]
        cands.sort(key=lambda k: np.linalg.norm(k.T_world[:3, 3] - T_world[:3, 3]))
        cands = cands[:self.p.max_candidates]
        closures = []
        if cands:
            inits = [rigid_inv(k.T_world) @ T_world for k in cands]
            results, classes, best = self.b.loop_closure(scan, [k.data for k in cands], inits,
                                                         self.p.new_keyframe_ratio)
            for k, r, c in zip(cands, results, classes):
                closures.append((k.id, int(c), r["inlier_ratio"]))
                if c == 1:  # weak: an edge between the current keyframe and the neighbour
                    self.edges.append(Edge(cur.id, k.id, T @ rigid_inv(r["T"]), EDGE_WEAK, r["inlier_ratio"]))
            if best >= 0:
                nk, r = cands[best], results[best]
                # cur -> neighbour through the sweep: T_cur_scan T_scan_nk
                T_cur_nk = T @ rigid_inv(r["T"])
                self.edges.append(Edge(cur.id, nk.id, T_cur_nk, EDGE_STRONG, r["inlier_ratio"]))
                removed = self.b.consistency(cur.data, nk.data, rigid_inv(T_cur_nk))
                self.current = nk.id
                self._set_last(r["T"], False)
                return Step("switched", nk.id, r["T"], nk.T_world @ r["T"], r["inlier_ratio"], closures, removed)
        # ---- no strong closure: the sweep becomes a keyframe
        nk = Keyframe(len(self.keyframes), T_world, self.b.new_keyframe(scan))
        self.keyframes.append(nk)
        self.edges.append(Edge(cur.id, nk.id, T, EDGE_ODOMETRY, ratio))
        removed = self.b.consistency(cur.data, nk.data, rigid_inv(T))
        self.current = nk.id
        self._set_last(np.eye(4), False)
        return Step("new_keyframe", nk.id, np.eye(4), T_world, ratio, closures, removed)


class GpuBackend:
    """The map's data steps on the GPU: surfels, registration, fusion, the
    batched loop-closure search (grid search + registration + classes) and
    the moving-object check, all through the C ABI."""

    def __init__(self, ctx, geom, icp=None, grid="default", fuse=None, consistency=None):
        import paper_2101_00585_amd as ups
        self.ups = ups
        self.ctx = ctx
        self.g = geom
        self.icp = icp or ups.IcpParams(levels=3, iters=(10, 10, 10), stop_update_norm=1e-6)
        self.grid = ups.GridParams() if grid == "default" else grid
        self.fuse_p = fuse or ups.FuseParams()
        self.cons = consistency or ups.ConsistencyParams()

    def normals(self, depth):
        torch = self.ups._torch()
        if not isinstance(depth, torch.Tensor):
            depth = torch.from_numpy(np.ascontiguousarray(depth, dtype=np.float32)).cuda(self.ctx.device)
        return self.ups.panorama_normals(self.ctx, self.g, depth)

    def new_keyframe(self, scan):
        torch = self.ups._torch()
        surf = scan.clone()
        count = (surf[..., 3] > 0).to(torch.int16).contiguous()
        return dict(surfel=surf, count=count)

    def register(self, scan, kf, init):
        r = self.ups.register_scan(self.ctx, self.g, scan, self.g, kf["surfel"], init, self.icp)
        return self.ups.read_result(r)

    def fuse(self, scan, kf, T):
        self.ups.fuse_scan(self.ctx, self.g, scan, self.g, kf["surfel"], kf["count"], T, self.fuse_p)

    def loop_closure(self, scan, kfs, inits, threshold):
        ups = self.ups
        torch = ups._torch()
        items = [dict(scan_geom=self.g, kf_geom=self.g, scan_surfel=scan, kf_surfel=kf["surfel"]) for kf in kfs]
        b = ups.Batch(self.ctx, items, self.icp)
        try:
            base = torch.stack([ups.pose_tensor(T, scan.device) for T in inits])
            if self.grid is not None:
                start, _, _ = b.grid_search(self.grid, base)
            else:
                start = base
            res = b.register(start)
            cls, best = ups.classify_loop_closures(self.ctx, res, threshold)
            torch.cuda.synchronize()
            return ups.read_results(res), cls.cpu().numpy(), int(best.cpu().numpy()[0])
        finally:
            b.close()

    def consistency(self, kf_a, kf_b, T_ba):
        _, _, removed = self.ups.keyframe_consistency(self.ctx, self.g, kf_a["surfel"], kf_a["count"], self.g,
                                                      kf_b["surfel"], kf_b["count"], T_ba, self.cons)
        return tuple(int(v) for v in removed.cpu().numpy())
