"""Training data, training loop and batched use of the learned pose proposal.

The network and its kernels live in the library (``Proposal``: BF16 MFMA
convolutions, FP32 head, Adam); this module feeds it.

Training pairs are rendered scan / keyframe panoramas of the synthetic room
and outdoor scenes with motions up to 30 deg yaw and 2 m.  Labels are what
the registration itself returns when started at the true motion (the
optimum of the method nearest the truth), so the network learns poses the
method generates.  Each rendered pair is reused many times under exact
symmetries of a panorama pair:

  * rolling the scan image alone by k2 columns rotates the scan frame by
    D2 = 2 pi k2 / 256 about its z axis:  T' = T Rz(D2) (this widens the
    relative yaw to about +-100 deg, the range of loop-closure candidates);
  * rolling both images by k columns is a rotation of both sensor frames by
    D = 2 pi k / 256 about z:  T' = Rz(D)^T T Rz(D);
  * mirroring both images in azimuth (column j -> -j) is the reflection
    S = diag(1, -1, 1) of both frames:  T' = S T S.

Run ``python -m paper_2101_00585_amd.proposal --help`` to train.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import (Batch, Context, IcpParams, Proposal, UpsError, load, pose_tensor, proposal_num_params,
               read_results)

PARAMS_FILE = os.path.join(os.path.dirname(__file__), "proposal_params.npy")
S_OMEGA, S_T = 0.25, 1.0  # output scales of the network (rad, m)
COLS = 256
SCAN_ROLL = 48  # scan-only rolls of up to +-48 columns (+-67.5 deg) in training
BATCH_ICP = dict(levels=3, iters=(10, 10, 10), stop_update_norm=1e-6)
MIN_INLIER_RATIO = 0.5  # below it a proposal-started registration is rerun from the identity


def _torch():
    import torch
    return torch


# ---------------------------------------------------------------- poses

def log_so3(R):
    """Rotation vector of a rotation matrix (angle below pi)."""
    R = np.asarray(R, dtype=np.float64)
    v = 0.5 * np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    s = float(np.linalg.norm(v))
    c = (float(np.trace(R)) - 1.0) / 2.0
    if s < 1e-12:
        return v
    return v * (math.atan2(s, c) / s)


def pose_to_target(T):
    """Network target y[6] of a scan -> keyframe pose."""
    T = np.asarray(T, dtype=np.float64)
    return np.concatenate([log_so3(T[:3, :3]) / S_OMEGA, T[:3, 3] / S_T])


def roll_targets(y, k):
    """Targets after rolling both images of each pair by k[b] columns: the
    rotation vector and translation turn by -2 pi k / 256 about z."""
    y = np.asarray(y, dtype=np.float64)
    a = -2.0 * math.pi * np.asarray(k, dtype=np.float64) / COLS
    c, s = np.cos(a), np.sin(a)
    out = y.copy()
    for o in (0, 3):
        out[:, o] = c * y[:, o] - s * y[:, o + 1]
        out[:, o + 1] = s * y[:, o] + c * y[:, o + 1]
    return out


def mirror_targets(y, flip):
    """Targets after mirroring both images of the flagged pairs in azimuth:
    with S = diag(1, -1, 1), S R S has rotation vector (-wx, wy, -wz) and
    S t = (tx, -ty, tz)."""
    y = np.asarray(y, dtype=np.float64).copy()
    f = np.asarray(flip, dtype=bool)
    y[f, 0] *= -1
    y[f, 2] *= -1
    y[f, 4] *= -1
    return y


def scan_roll_targets(y, k2):
    """Targets after rolling the scan image alone by k2[b] columns: T' = T Rz(2 pi k2 / 256)."""
    y = np.asarray(y, dtype=np.float64)
    out = y.copy()
    for b in range(y.shape[0]):
        R = _exp_so3(y[b, :3] * S_OMEGA)
        a = 2.0 * math.pi * float(k2[b]) / COLS
        Rz = np.array([[math.cos(a), -math.sin(a), 0.0], [math.sin(a), math.cos(a), 0.0], [0.0, 0.0, 1.0]])
        out[b, :3] = log_so3(R @ Rz) / S_OMEGA
    return out


def _exp_so3(w):
    th = float(np.linalg.norm(w))
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + math.sin(th) / th * K + (1 - math.cos(th)) / th ** 2 * K @ K


def augment_inputs(x, k, flip, k2=None):
    """Roll each pair's scan image alone by k2[b] columns (if given), then both
    images by k[b] columns (x'[..., j, :] = x[..., (j + k) mod 256, :]), then
    mirror the flagged pairs (j -> -j mod 256).  x: device bfloat16
    [n, 32, 256, 2]; k, k2: int64 [n]; flip: bool [n]."""
    torch = _torch()
    n = x.shape[0]
    j = torch.arange(COLS, device=x.device)
    if k2 is not None:
        i2 = ((j[None, :] + k2[:, None]) % COLS)[:, None, :].expand(n, x.shape[1], COLS)
        scan = torch.gather(x[..., 1], 2, i2)
        x = torch.stack([x[..., 0], scan], dim=3)
    idx = (j[None, :] + k[:, None]) % COLS
    idx = torch.where(flip[:, None], idx.gather(1, (COLS - j[None, :].expand_as(idx)) % COLS), idx)
    idx = idx[:, None, :, None].expand(n, x.shape[1], COLS, x.shape[3])
    return torch.gather(x, 2, idx)


# ---------------------------------------------------------------- data

def _pair_items(pairs, dev):
    torch = _torch()
    items = []
    for p in pairs:
        g = p["geom"]
        items.append(dict(scan_geom=g, kf_geom=g, scan_depth=torch.from_numpy(p["scan"]).to(dev),
                          kf_depth=torch.from_numpy(p["kf"]).to(dev),
                          scan_surfel=torch.empty((g.rows, g.cols, 4), dtype=torch.float32, device=dev),
                          kf_surfel=torch.empty((g.rows, g.cols, 4), dtype=torch.float32, device=dev)))
    return items


def build_dataset(ctx, prop, pairs, chunk=256, log=None):
    """(x [n, 32, 256, 2] bfloat16 device inputs, y [n, 6] targets, keep mask)
    for rendered pairs: surfels and the method's labels on the GPU (batched
    registration started at the true motion), inputs by the proposal's input
    kernel.  Pairs whose registration from the truth fails or moves more
    than 2 deg / 0.1 m from it are dropped (keep mask)."""
    torch = _torch()
    dev = torch.device("cuda")
    xs, ys, keep = [], [], []
    for c0 in range(0, len(pairs), chunk):
        part = pairs[c0:c0 + chunk]
        items = _pair_items(part, dev)
        b = Batch(ctx, items, IcpParams(**BATCH_ICP))
        b.normals()
        res = read_results(b.register([p["T_gt"] for p in part]))
        b.close()
        prop.plan_input([it["kf_surfel"] for it in items], [it["scan_surfel"] for it in items],
                        [it["kf_geom"] for it in items], [it["scan_geom"] for it in items])
        x = torch.empty((len(part), 32, COLS, 2), dtype=torch.bfloat16, device=dev)
        prop.input(x)
        torch.cuda.synchronize()
        for r, p in zip(res, part):
            dT = np.linalg.inv(p["T_gt"]) @ r["T"]
            ang = float(np.linalg.norm(log_so3(dT[:3, :3])))
            ok = r["status"] in (0, 1) and ang < math.radians(2.0) and np.linalg.norm(dT[:3, 3]) < 0.1
            keep.append(ok)
            ys.append(pose_to_target(r["T"]))
        xs.append(x)
        if log:
            log(f"labelled {min(c0 + chunk, len(pairs))}/{len(pairs)} pairs")
    return torch.cat(xs), np.array(ys), np.array(keep)


def _render_chunk(job):
    """Training pairs c0..c1-1 (seeds base_seed + k): yaw up to 30 deg,
    translation up to 2 m, 64x512 or 128x1024."""
    c0, c1, base_seed = job
    from synth import workloads as W
    return [W.batch_pair(k, base_seed=base_seed, max_angle=math.radians(30.0), max_trans=2.0,
                         sizes=((64, 512), (128, 1024))) for k in range(c0, c1)]


def _render_worker_init():
    import synth
    synth.DEFAULT_THREADS = 1  # one ray-casting thread per worker process


def labelled_inputs(ctx, prop, n, base_seed, chunk=256, log=None, pool=None):
    """build_dataset over n pairs rendered chunk by chunk (only the 32x256
    network inputs and the labels are kept, so the full-resolution renders
    of a large training set never sit in memory together).  pool: a process
    pool (created before the GPU is touched) that renders chunks ahead."""
    torch = _torch()
    xs, ys, keeps = [], [], []
    t0 = time.perf_counter()
    jobs = [(c0, min(n, c0 + chunk), base_seed) for c0 in range(0, n, chunk)]
    chunks = pool.imap(_render_chunk, jobs) if pool is not None else map(_render_chunk, jobs)
    for (c0, _, _), pairs in zip(jobs, chunks):
        x, y, keep = build_dataset(ctx, prop, pairs, chunk=chunk)
        xs.append(x)
        ys.append(y)
        keeps.append(keep)
        if log and (c0 // chunk) % 20 == 19:
            log(f"rendered and labelled {min(n, c0 + chunk)}/{n} pairs ({time.perf_counter() - t0:.0f} s)")
    return torch.cat(xs), np.concatenate(ys), np.concatenate(keeps)


def init_params(seed=0):
    """He-normal convolution weights, zero biases, a small output layer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    layers = ((2, 32), (32, 64), (64, 96), (96, 128), (128, 128))
    for cin, cout in layers:
        parts += [rng.normal(size=9 * cin * cout) * math.sqrt(2.0 / (9 * cin)), np.zeros(cout)]
    feat = 2 * 16 * 128
    parts += [rng.normal(size=6 * feat) * math.sqrt(1.0 / feat) * 0.1, np.zeros(6)]
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == proposal_num_params()
    return p


def _loop_state_path(checkpoint):
    return checkpoint + ".loop.npz"


def train(prop, x, y, steps=6000, batch=256, lr=1e-3, seed=1, val=None, log=None, every=500, checkpoint=None,
          checkpoint_every=1000, resume=False, until=None):
    """Adam on augmented batches drawn from (x, y); cosine-decayed learning
    rate after a short warm-up.  val = {name: (x_val, y_val)} for periodic
    error reports.  With ``checkpoint`` (a path), every ``checkpoint_every``
    steps the network's checkpoint (parameters, Adam moments and step count)
    goes to that path and the loop's state (the next step and the batch
    generator's state) beside it; ``resume`` continues from them, taking the
    same batches and learning rates as the uninterrupted run.  ``until``
    stops before that step (the schedule still spans ``steps``).  Returns the
    loss history (of this call)."""
    torch = _torch()
    dev = x.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    start = 0
    if resume:
        prop.load_checkpoint(checkpoint)
        st = np.load(_loop_state_path(checkpoint))
        start = int(st["step"])
        gen.set_state(torch.from_numpy(st["rng"]))
    yt = torch.from_numpy(np.asarray(y, dtype=np.float64)).to(dev)
    n = x.shape[0]
    losses = []
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    for s in range(start, steps if until is None else min(until, steps)):
        idx = torch.randint(0, n, (batch,), device=dev, generator=gen)
        k = torch.randint(0, COLS, (batch,), device=dev, generator=gen)
        k2 = torch.randint(-SCAN_ROLL, SCAN_ROLL + 1, (batch,), device=dev, generator=gen)
        flip = torch.randint(0, 2, (batch,), device=dev, generator=gen).bool()
        xb = augment_inputs(x[idx], k, flip, k2).contiguous()
        yb = _augment_targets_torch(yt[idx], k, flip, k2).float().contiguous()
        warm = min(1.0, (s + 1) / 200.0)
        cur = lr * warm * (0.01 + 0.99 * 0.5 * (1 + math.cos(math.pi * s / steps)))
        prop.train_step(xb, yb, cur, loss)
        if checkpoint and (s + 1) % checkpoint_every == 0:
            prop.save_checkpoint(checkpoint)
            np.savez(_loop_state_path(checkpoint), step=np.int64(s + 1), rng=gen.get_state().numpy())
        if (s + 1) % 50 == 0:
            losses.append((s + 1, float(loss.item())))
        if log and ((s + 1) % every == 0 or s + 1 == steps):
            msg = f"step {s + 1}/{steps} loss {losses[-1][1]:.4f} lr {cur:.2e} ({time.perf_counter() - t0:.0f} s)"
            for name, (xv, yv) in (val or {}).items():
                e = evaluate(prop, xv, yv)
                msg += f"  {name}: rot {e['rot_deg_median']:.2f} deg, trans {e['trans_m_median']:.3f} m"
            log(msg)
    return losses


def _exp_so3_t(w):
    torch = _torch()
    th = torch.linalg.norm(w, dim=1).clamp_min(1e-12)[:, None, None]
    K = torch.zeros(w.shape[0], 3, 3, dtype=w.dtype, device=w.device)
    K[:, 0, 1], K[:, 0, 2], K[:, 1, 2] = -w[:, 2], w[:, 1], -w[:, 0]
    K[:, 1, 0], K[:, 2, 0], K[:, 2, 1] = w[:, 2], -w[:, 1], w[:, 0]
    eye = torch.eye(3, dtype=w.dtype, device=w.device).expand_as(K)
    return eye + torch.sin(th) / th * K + (1 - torch.cos(th)) / th ** 2 * (K @ K)


def _log_so3_t(R):
    torch = _torch()
    v = 0.5 * torch.stack([R[:, 2, 1] - R[:, 1, 2], R[:, 0, 2] - R[:, 2, 0], R[:, 1, 0] - R[:, 0, 1]], dim=1)
    s = torch.linalg.norm(v, dim=1)
    c = (R[:, 0, 0] + R[:, 1, 1] + R[:, 2, 2] - 1.0) / 2.0
    f = torch.where(s > 1e-12, torch.atan2(s, c) / s.clamp_min(1e-12), torch.ones_like(s))
    return v * f[:, None]


def _augment_targets_torch(y, k, flip, k2=None):
    torch = _torch()
    if k2 is not None:
        a2 = 2.0 * math.pi * k2.double() / COLS
        Rz = torch.zeros(y.shape[0], 3, 3, dtype=torch.float64, device=y.device)
        Rz[:, 0, 0], Rz[:, 0, 1], Rz[:, 1, 0], Rz[:, 1, 1] = torch.cos(a2), -torch.sin(a2), torch.sin(a2), torch.cos(a2)
        Rz[:, 2, 2] = 1.0
        y = y.clone()
        y[:, :3] = _log_so3_t(_exp_so3_t(y[:, :3] * S_OMEGA) @ Rz) / S_OMEGA
    a = -2.0 * math.pi * k.double() / COLS
    c, s = torch.cos(a), torch.sin(a)
    out = y.clone()
    for o in (0, 3):
        out[:, o] = c * y[:, o] - s * y[:, o + 1]
        out[:, o + 1] = s * y[:, o] + c * y[:, o + 1]
    sign = torch.ones_like(out)
    sign[:, 0] = sign[:, 2] = sign[:, 4] = -1.0
    return torch.where(flip[:, None], out * sign, out)


def evaluate(prop, x, y, chunk=None):
    """Median rotation (deg) and translation (m) errors of the proposed
    increments against the targets."""
    torch = _torch()
    chunk = chunk or prop.max_batch
    outs = []
    for c0 in range(0, x.shape[0], chunk):
        xb = x[c0:c0 + chunk].contiguous()
        outs.append(prop.forward(xb.shape[0], xb).double().cpu().numpy())
    out = np.concatenate(outs)
    y = np.asarray(y)
    rot = np.degrees(np.linalg.norm((out[:, :3] - y[:, :3]) * S_OMEGA, axis=1))
    tr = np.linalg.norm((out[:, 3:] - y[:, 3:]) * S_T, axis=1)
    return dict(rot_deg_median=float(np.median(rot)), trans_m_median=float(np.median(tr)),
                rot_deg_p90=float(np.percentile(rot, 90)), trans_m_p90=float(np.percentile(tr, 90)))


def load_params(path=PARAMS_FILE):
    if not os.path.exists(path):
        raise UpsError(f"no trained proposal parameters at {path}")
    p = np.load(path, allow_pickle=False).astype(np.float32)
    if p.size != proposal_num_params():
        raise UpsError("proposal parameter file does not match the network")
    return p


# ------------------------------------------------------ batched use

class ProposedRegistration:
    """A batch of registrations started from the network's proposals, with
    the identity-started fallback for those whose inlier ratio stays below
    ``min_inlier_ratio``.  ``run`` enqueues only kernels (input, network,
    poses, registration, fallback), so it can be captured in a HIP graph.
    The proposal holds one planned input: a later ProposedRegistration (or
    plan_input) on the same Proposal replaces this one's.  The scan channel
    is read from an item's ``scan_depth`` when it has one (the same valid
    ranges as its surfels' range channel, 4 bytes per sample instead of a
    16-byte surfel), else from ``scan_surfel``."""

    def __init__(self, ctx: Context, prop: Proposal, batch: Batch, items, min_inlier_ratio=MIN_INLIER_RATIO,
                 start_level=None):
        torch = _torch()
        self.batch, self.prop, self.n = batch, prop, len(items)
        # the proposal-started registrations run the batch's schedule from
        # `start_level` down (the coarser levels left out); the fallback keeps
        # the full schedule
        full = list(batch.params.iters)[:batch.params.levels]
        if start_level is None:
            start_level = len(full) - 1
        if not 0 <= start_level < len(full):
            raise UpsError("start_level must be one of the batch's pyramid levels")
        self.full_iters = full
        self.start_iters = [it if l <= start_level else 0 for l, it in enumerate(full)]
        if self.n > prop.max_batch:
            raise UpsError("batch larger than the proposal's max_batch")
        self.rho = float(min_inlier_ratio)
        prop.plan_input([it["kf_surfel"] for it in items],
                        [it["scan_depth"] if it.get("scan_depth") is not None else it["scan_surfel"] for it in items],
                        [it["kf_geom"] for it in items], [it["scan_geom"] for it in items])
        self.y = torch.empty((self.n, 6), dtype=torch.float32, device="cuda")
        self.poses = torch.empty((self.n, 12), dtype=torch.float64, device="cuda")
        self.count = torch.zeros(1, dtype=torch.int32, device="cuda")

    def run(self, results):
        """The whole path, fallback launches always enqueued (capturable)."""
        self.propose_and_register(results)
        self.batch.fallback_run(results)
        return results

    def propose_and_register(self, results):
        """Everything up to the fallback decision: network input, network,
        poses, registration from them, and the fallback plan (the number of
        registrations to rerun lands in ``self.count``)."""
        self.prop.input()
        self.prop.forward(self.n, None, self.y)
        self.prop.poses(self.y, self.poses)
        if self.start_iters != self.full_iters:
            self.batch.set_iterations(self.start_iters)
            try:
                self.batch.register(self.poses, results)
            finally:
                self.batch.set_iterations(self.full_iters)
        else:
            self.batch.register(self.poses, results)
        self.batch.fallback_plan(results, self.rho, self.count)
        return results

    def run_checked(self, results):
        """propose_and_register, then the fallback only if some registration
        needs it (one host read of the count)."""
        self.propose_and_register(results)
        if int(self.count.item()) > 0:
            self.batch.fallback_run(results)
        return results


# ---------------------------------------------------------------- CLI

def main(argv=None):
    ap = argparse.ArgumentParser(description="train the pose-proposal network on rendered pairs")
    ap.add_argument("--pairs", type=int, default=4000, help="rendered training pairs")
    ap.add_argument("--val-pairs", type=int, default=256)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=PARAMS_FILE)
    ap.add_argument("--log-json", default=None)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="processes that render training pairs")
    ap.add_argument("--checkpoint", default=None, help="training checkpoint path (written every 1000 steps)")
    ap.add_argument("--resume", action="store_true", help="continue from --checkpoint")
    a = ap.parse_args(argv)

    def log(m):
        print(f"[train] {m}", file=sys.stderr, flush=True)

    # the rendering workers are forked before anything touches the GPU
    pool = None
    if a.workers > 1:
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(a.workers, initializer=_render_worker_init)
    torch = _torch()
    load()
    log(f"rendering and labelling {a.pairs} training pairs and {a.val_pairs} validation pairs")
    ctx = Context(0, max_pixels=128 * 2048, max_batch=256, max_batch_pixels=256 * 128 * 2048)
    prop = Proposal(ctx, max(a.batch, 256))
    x, y, keep = labelled_inputs(ctx, prop, a.pairs, 1_000_000, log=log, pool=pool)
    xv, yv, kv = labelled_inputs(ctx, prop, a.val_pairs, 3_000_000, log=log, pool=pool)
    if pool is not None:
        pool.close()
        pool.join()
    kt = torch.from_numpy(keep).to(x.device)
    x, y = x[kt].contiguous(), y[keep]
    xv, yv = xv[torch.from_numpy(kv).to(xv.device)].contiguous(), yv[kv]
    log(f"kept {keep.sum()}/{keep.size} training and {kv.sum()}/{kv.size} validation pairs")
    # validation with the scan rolled as in training (relative yaw up to ~100 deg)
    g = torch.Generator(device=xv.device)
    g.manual_seed(12345)
    k2v = torch.randint(-SCAN_ROLL, SCAN_ROLL + 1, (xv.shape[0],), device=xv.device, generator=g)
    zero = torch.zeros_like(k2v)
    nof = torch.zeros_like(k2v, dtype=torch.bool)
    xw = augment_inputs(xv, zero, nof, k2v).contiguous()
    yw = _augment_targets_torch(torch.from_numpy(yv).to(xv.device), zero, nof, k2v).cpu().numpy()
    val = {"val": (xv, yv), "val wide yaw": (xw, yw)}
    prop.set_params(init_params(a.seed))
    t0 = time.perf_counter()
    losses = train(prop, x, y, steps=a.steps, batch=a.batch, lr=a.lr, seed=a.seed + 1, val=val, log=log,
                   checkpoint=a.checkpoint, resume=a.resume)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    ev = {name: evaluate(prop, *v) for name, v in val.items()}
    np.save(a.out, prop.get_params())
    log(f"trained {a.steps} steps in {secs:.1f} s; validation {ev}; saved {a.out}")
    if a.log_json:
        with open(a.log_json, "w") as f:
            json.dump(dict(args=vars(a), seconds=secs, validation=ev, losses=losses,
                           kept=[int(keep.sum()), int(keep.size)]), f, indent=1)
    prop.close()
    ctx.close()


if __name__ == "__main__":
    main()
