"""Per-layer timing of the pose-proposal network's convolutions.

For each of the five 3x3 convolutions at the network's shapes (a batch of
panoramas of 32 x 256, channels 2-32-64-96-128-128, strides 2, 2, 2, 2, 1),
times the forward pass, the data gradient and the weight gradient through the
library's layer entry points, each replayed from a HIP graph of `reps`
launches, and prints microseconds and TFLOP/s (2 x output pixels x 9 cin x
cout multiply-adds per pass) against the 2.5 PFLOP/s dense BF16 peak of an
MI355X.

    python -m paper_2101_00585_amd.conv_bench [--batch 256] [--reps 50]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BF16_PEAK_TFLOPS = 2500.0
ROWS, COLS = 32, 256
CIN = (2, 32, 64, 96, 128)
COUT = (32, 64, 96, 128, 128)
STRIDE = (2, 2, 2, 2, 1)


def layer_shapes(batch: int):
    h, w = ROWS, COLS
    out = []
    for cin, cout, s in zip(CIN, COUT, STRIDE):
        out.append(dict(n=batch, h=h, w=w, cin=cin, cout=cout, stride=s))
        h, w = (h - 1) // s + 1, (w - 1) // s + 1
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--reps", type=int, default=50)
    ap.add_argument("--json", action="store_true", help="one JSON line per layer instead of a table")
    args = ap.parse_args(argv)
    import torch
    import paper_2101_00585_amd as ups

    lib = ups.load()
    dev = torch.device("cuda:0")
    g = torch.Generator(device="cpu").manual_seed(7)
    stream = torch.cuda.Stream()
    rows = []
    for k, c in enumerate(layer_shapes(args.batch)):
        n, h, w, cin, cout, s = c["n"], c["h"], c["w"], c["cin"], c["cout"], c["stride"]
        ho, wo = (h - 1) // s + 1, (w - 1) // s + 1
        x = torch.randn((n, h, w, cin), generator=g).to(torch.bfloat16).to(dev)
        w_nk = (0.1 * torch.randn((cout, 9 * cin), generator=g)).to(torch.bfloat16).to(dev)
        w_kn = w_nk.t().contiguous()
        b = (0.1 * torch.randn(cout, generator=g)).to(dev)
        y = ups.conv3x3_forward(x, w_nk, b, cout, s)
        dy = torch.randn((n, ho, wo, cout), generator=g).to(dev)
        dx = torch.empty((n, h, w, cin), dtype=torch.float32, device=dev)
        work_n = int(lib.ups_conv3x3_backward_weight_work(n, h, w, cin, cout, s))
        work = torch.empty(max(work_n, 1), dtype=torch.float32, device=dev)
        dw = torch.empty((9 * cin, cout), dtype=torch.float32, device=dev)
        db = torch.empty(cout, dtype=torch.float32, device=dev)
        p = ups._P
        passes = {
            "forward": lambda: lib.ups_conv3x3_forward(n, h, w, cin, cout, s, p(x.data_ptr()), p(w_nk.data_ptr()),
                                                       p(b.data_ptr()), p(y.data_ptr()), ups._stream()),
            "backward_data": lambda: lib.ups_conv3x3_backward_data(n, h, w, cin, cout, s, p(y.data_ptr()),
                                                                   p(dy.data_ptr()), p(w_kn.data_ptr()),
                                                                   p(dx.data_ptr()), ups._stream()),
            "backward_weight": lambda: lib.ups_conv3x3_backward_weight(n, h, w, cin, cout, s, p(x.data_ptr()),
                                                                       p(y.data_ptr()), p(dy.data_ptr()),
                                                                       p(dw.data_ptr()), p(db.data_ptr()),
                                                                       p(work.data_ptr()), work_n, ups._stream()),
        }
        flops = 2.0 * n * ho * wo * 9 * cin * cout
        for name, fn in passes.items():
            with torch.cuda.stream(stream):
                for _ in range(3):
                    ups._check(fn())
                torch.cuda.synchronize()
                graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(graph, stream=stream):
                    for _ in range(args.reps):
                        ups._check(fn())
                graph.replay()
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                best = float("inf")
                for _ in range(5):
                    e0.record(stream)
                    graph.replay()
                    e1.record(stream)
                    e1.synchronize()
                    best = min(best, e0.elapsed_time(e1) * 1e3 / args.reps)
            tf = flops / (best * 1e-6) / 1e12
            rows.append(dict(layer=k + 1, pass_=name, n=n, h=h, w=w, cin=cin, cout=cout, stride=s,
                             us=round(best, 3), gflop=round(flops / 1e9, 4), tflops=round(tf, 2),
                             frac=round(tf / BF16_PEAK_TFLOPS, 5)))
    if args.json:
        for r in rows:
            print(json.dumps(r))
    else:
        print(f"{'layer':>5} {'pass':>16} {'shape (n,h,w,cin->cout,s)':>30} {'us':>9} {'GFLOP':>8} {'TFLOP/s':>8} "
              f"{'of peak':>8}")
        for r in rows:
            shape = f"{r['n']},{r['h']},{r['w']},{r['cin']}->{r['cout']},s{r['stride']}"
            print(f"{r['layer']:>5} {r['pass_']:>16} {shape:>30} {r['us']:>9.2f} {r['gflop']:>8.3f} "
                  f"{r['tflops']:>8.1f} {100 * r['frac']:>7.2f}%")
        tot_us = sum(r["us"] for r in rows)
        tot_gf = sum(r["gflop"] for r in rows)
        print(f"all 15 passes: {tot_us:.1f} us, {tot_gf:.2f} GFLOP, {tot_gf / tot_us * 1e3:.1f} TFLOP/s")
    return 0


if __name__ == "__main__":
    sys.exit(main())
