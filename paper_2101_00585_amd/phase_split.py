"""Per-launch phase split of the sensor-scale single registration.

Loads the instrumented library (`python -m paper_2101_00585_amd.build
--phases` writes libupslam_phases.so: the same kernels plus real-time clock
marks), registers the 128x1024 outdoor scan against its keyframe fused from
ten scans (3 levels, 10 iterations each) from a HIP graph, and prints for
every Gauss-Newton iteration and the evaluation launch, in microseconds (100
MHz clock, mean over `reps` replays); the iterations of a level that runs in
one launch (the one-XCD level kernel) are timed like separate launches:
  gap       the previous iteration's last block exit to this one's first
            entry (a launch gap, or the level kernel's exchange between
            iterations)
  partials  tile 0: entry to the previous launch's partials and state reduced
  solve     tile 0: the FP64 solve and pose update (thread 0)
  pixels    tile 0: its pixels (association, terms, per-thread sums)
  store     tile 0: the block partial (and the wait for the block's slowest wavefront)
  tail      tile 0's partial stored to the launch's last block exit
  total     first entry to last exit

    python -m paper_2101_00585_amd.phase_split [--reps 5]
"""
from __future__ import annotations

import argparse
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

LAUNCHES = 64


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    import numpy as np
    import torch

    import paper_2101_00585_amd as ups
    from paper_2101_00585_amd import build as B
    from synth import workloads as W

    if not os.path.exists(B.SO_PHASES):
        raise SystemExit(f"{B.SO_PHASES} is not built: run `python -m paper_2101_00585_amd.build --phases`")
    ups._SO = B.SO_PHASES
    lib = ups.load()
    lib.ups_debug_phase_read.argtypes = [ctypes.c_void_p]
    lib.ups_debug_phase_read.restype = ctypes.c_int
    c1 = W.config1()
    g = c1["geom"]
    dev = torch.device("cuda:0")
    ctx = ups.Context(0, max_pixels=g.rows * g.cols)
    kf = torch.zeros((g.rows, g.cols, 4), dtype=torch.float32, device=dev)
    cnt = torch.zeros((g.rows, g.cols), dtype=torch.int16, device=dev)
    tmp = torch.empty_like(kf)
    for d, T in zip(c1["kf_scans"], c1["T_kf_scans"]):
        ups.panorama_normals(ctx, g, torch.from_numpy(d).to(dev), tmp)
        ups.fuse_scan(ctx, g, tmp, g, kf, cnt, T)
    scan = ups.panorama_normals(ctx, g, torch.from_numpy(c1["scan"]).to(dev))
    init = ups.pose_tensor(c1["T_init"], dev)
    res = ups.new_result(dev)
    params = ups.IcpParams(levels=3, iters=(10, 10, 10))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for _ in range(3):
            ups.register_scan(ctx, g, scan, g, kf, init, params, res)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            ups.register_scan(ctx, g, scan, g, kf, init, params, res)
    buf = np.zeros(LAUNCHES * 7, dtype=np.uint64)
    runs = []
    for rep in range(args.reps + 1):
        torch.cuda.synchronize()
        ups._check(lib.ups_debug_phase_read(buf.ctypes.data))  # reset
        graph.replay()
        torch.cuda.synchronize()
        ups._check(lib.ups_debug_phase_read(buf.ctypes.data))
        if rep > 0:
            runs.append(buf.astype(np.float64).copy())
    a = np.array(runs)
    marks = a[:, :LAUNCHES * 5].reshape(len(runs), LAUNCHES, 5)
    first = a[:, LAUNCHES * 5:LAUNCHES * 6]
    last = a[:, LAUNCHES * 6:]
    n = sum(params.iters) + 1
    us = 1.0 / 100.0  # 100 MHz ticks -> us
    rows = []
    for i in range(n):
        gap = (first[:, i] - last[:, i - 1]) * us if i else np.zeros(len(runs))
        d = lambda p, q: ((marks[:, i, q] - marks[:, i, p]) * us).mean()
        rows.append(dict(launch=i, gap=gap.mean(), partials=d(0, 1), solve=d(1, 2), pixels=d(2, 3), store=d(3, 4),
                         tail=((last[:, i] - marks[:, i, 4]) * us).mean(), total=((last[:, i] - first[:, i]) * us).mean()))
    names = ["launch", "gap", "partials", "solve", "pixels", "store", "tail", "total"]
    print("  ".join(f"{c:>8}" for c in names))
    for r in rows:
        label = f"L{2 - r['launch'] // 10}/{r['launch'] % 10}" if r["launch"] < 30 else "eval"
        print(f"{label:>8}  " + "  ".join(f"{r[c]:8.2f}" for c in names[1:]))
    for lvl in (2, 1, 0):
        sel = [r for r in rows[1:30] if 2 - r["launch"] // 10 == lvl]
        print(f"level {lvl} mean: " + "  ".join(f"{c} {np.mean([r[c] for r in sel]):.2f}" for c in names[1:]))
    span = ((last[:, n - 1] - first[:, 0]) * us).mean()
    print(f"first entry of launch 0 to last exit of the evaluation launch: {span:.1f} us")
    return 0


if __name__ == "__main__":
    sys.exit(main())
