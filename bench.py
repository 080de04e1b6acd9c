#!/usr/bin/env python3
"""Throughput of the depth path on one MI355X.

A step is one pass of the whole path over one synthetic 1280x720 pair with
D = 128 and 8 aggregation paths: IR noise applied to both clean images
(Sec. VI-C), census, aggregation, winner/uniqueness/sub-pixel/LR selection,
median and depth (Sec. VI-D).  Inputs (clean images and noise draws) are
resident in HBM before timing starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic work of the aggregation pass per (pixel, disparity, path):
# XOR + popcount for the matching cost, then min(d-1, d+1), +P1, min with L(d),
# min with P2, +C, -m and the running minimum of the path minimum m.
AGG_OPS_PER_PDR = 9
# MI355X: 256 CUs x 64 32-bit VALU lanes per clock x 2.4 GHz
VALU_PEAK_OPS = 256 * 64 * 2.4e9
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=720,
                    help="rows of the 1280x720 pair the oracle times (full pair = 720)")
    return ap.parse_args()


def cpu_baseline(params, left, right, rows):
    """The oracle as it stands, one host thread, on a bounded sample of the workload."""
    from oracle import oracle as orc
    orc.build(force=False)
    p = dict(params, height=rows)
    t0 = time.perf_counter()
    orc.sgm(p, np.ascontiguousarray(left[:rows]), np.ascontiguousarray(right[:rows]))
    dt = time.perf_counter() - t0
    frac = rows / params["height"]
    return {"value": round(frac / dt, 6), "unit": "pairs/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows} of 720 rows of one 1280x720 D=128 8-path pair (full path, census..depth), "
                      f"{dt:.2f} s single-threaded, scaled to pairs/s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2201_11924_amd.native as nat
    from synth import CONFIGS, make_pair, pair_seed

    cfg = CONFIGS["c1"]
    params = cfg["params"]
    W, H, D, P = params["width"], params["height"], params["max_disp"], params["num_paths"]
    pair = make_pair(cfg["spec"], pair_seed(1, 0))
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    cl, cr = t(pair.left), t(pair.right)
    gl, nl, gr, nr = t(pair.gamma_l), t(pair.n_l), t(pair.gamma_r), t(pair.n_r)
    L = torch.empty_like(cl)
    R = torch.empty_like(cr)
    depth = torch.empty((H, W), dtype=torch.float32, device=dev)
    disp = torch.empty_like(depth)
    flags = torch.empty((H, W), dtype=torch.uint8, device=dev)
    ss = nat.SimSense(params)

    def step():
        nat.ir_noise(cl, gl, nl, out=L)
        nat.ir_noise(cr, gr, nr, out=R)
        ss.compute(L, R, depth, disp, flags)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ss.profile(True)
    ss.profile_read()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        step()
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(end)
    calls, pass_ms = ss.profile_read()
    ss.profile(False)
    ms_step = ms_total / args.steps
    pairs_s = 1000.0 / ms_step
    vol = W * H * D

    agg_s = pass_ms["aggregate"] / calls / 1000.0
    agg_ops = AGG_OPS_PER_PDR * P * vol
    achieved = agg_ops / agg_s
    roofline = {"kernel": "aggregate_kernel", "bound": "alu", "achieved": round(achieved / 1e12, 3),
                "peak": round(VALU_PEAK_OPS / 1e12, 3), "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_OPS, 4),
                "traffic": None,
                "ops_per_launch": agg_ops, "avg_launch_us": round(agg_s * 1e6, 2)}
    out = {
        "metric": "stereo pairs/sec & Mpix·disp/s at 1280×720 D=128: 8-path SGM vs 2-path+net",
        "value": round(pairs_s, 2), "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "plain 8-path SGM, one 1280x720 pair, D=128, census 7x9 CS, P1=7 P2=86, "
                               "uniqueness 10%, LR 1 px, median 3x3, f=920 px, B=0.055 m",
                   "width": W, "height": H, "max_disp": D, "num_paths": P},
        "mpix_disp_per_s": round(vol * pairs_s / 1e6, 1),
        "pass_us": {k: round(v / calls * 1000.0, 2) for k, v in pass_ms.items()},
        "wall_s": round(wall, 3),
        "roofline": roofline,
    }
    ss.close()
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        Lh = orc.ir_noise(pair.left, pair.gamma_l, pair.n_l)
        Rh = orc.ir_noise(pair.right, pair.gamma_r, pair.n_r)
        out["cpu_baseline"] = cpu_baseline(params, Lh, Rh, args.cpu_sample_rows)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
