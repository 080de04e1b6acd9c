"""Fixed GPU workloads for profilers (rocprofv3 kernel traces and counters).

Each workload builds its seeded synthetic inputs, runs the library a few times
and prints one line; run it under a profiler, for example

    rocprofv3 --kernel-trace --stats -d OUT -o run -- \\
        python3 paper_2201_11924_amd/workloads.py pair --paths 8

Workloads:
  pair          one 1280x720 pair, D = 128, `--paths` 2/4/8, `--reps` compute calls
  batch         `--pairs` copies of one 1280x720 pair as plain 8-path and as the
                learned 2-path+net form (`--forms` both/learned/plain), one graph
                launch each per repetition
  net           fused inference of the learned net on `--pairs` 1280x720 feature maps
  train         `--reps` training steps of the learned net on a batch of `--pairs`
                640x480 feature maps (the training workload's batch shape)
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CHECKPOINT = os.path.join(ROOT, "paper_2201_11924_amd", "weights", "surrogate_640x480_d128.ckpt")


def _pair(nat, torch):
    from synth import CONFIGS, make_pair
    cfg = CONFIGS["pair_1280x720_d128"]
    pr = make_pair(cfg["spec"], 1_000_000)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    L = nat.ir_noise(t(pr.left), t(pr.gamma_l), t(pr.n_l))
    R = nat.ir_noise(t(pr.right), t(pr.gamma_r), t(pr.n_r))
    return cfg["params"], L, R


def run_pair(nat, torch, args):
    params, L, R = _pair(nat, torch)
    ss = nat.SimSense(dict(params, num_paths=args.paths))
    for _ in range(args.reps):
        ss(L, R)
    torch.cuda.synchronize()
    ss.close()
    return f"pair paths={args.paths} reps={args.reps}"


def run_batch(nat, torch, args):
    from paper_2201_11924_amd.train import load_checkpoint
    params8, L, R = _pair(nat, torch)
    params2 = dict(params8, num_paths=2)
    n = args.pairs
    Ls = [L.clone() for _ in range(n)]
    Rs = [R.clone() for _ in range(n)]
    W, H = params8["width"], params8["height"]
    net = nat.Net(16 * W * H, seed=0)
    if os.path.exists(CHECKPOINT):
        load_checkpoint(CHECKPOINT, net)
    b2 = nat.Batch([params2] * n)
    o2 = b2.outputs()
    unc = torch.zeros(n, dtype=torch.int32, device="cuda")
    b8 = nat.Batch([params8] * n) if args.forms in ("both", "plain") else None
    o8 = b8.outputs() if b8 else None
    res = []
    forms = [("learned", lambda: b2.learned_compute(net, Ls, Rs, o2, 0.5, unc)),
             ("plain8", lambda: b8.compute(Ls, Rs, o8))]
    for name, f in forms:
        if args.forms not in ("both", name.rstrip("8")):
            continue
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.reps):
            f()
        torch.cuda.synchronize()
        res.append(f"{name} {(time.perf_counter() - t0) / args.reps / n * 1000:.4f} ms/pair")
    b2.close()
    if b8:
        b8.close()
    net.close()
    return f"batch pairs={n}: " + ", ".join(res)


def run_net(nat, torch, args):
    B, H, W = args.pairs, 720, 1280
    rng = np.random.default_rng(0)
    x = np.zeros((B, H, W, 8), np.float32)
    x[..., :4] = rng.uniform(0, 1, (B, H, W, 4)).astype(np.float32)
    bits = (x.view(np.uint32) >> 16).astype(np.uint16)
    f = torch.from_numpy(bits).cuda().view(torch.int16)
    net = nat.Net(16, seed=1)
    if os.path.exists(CHECKPOINT):
        from paper_2201_11924_amd.train import load_checkpoint
        load_checkpoint(CHECKPOINT, net)
    d2 = torch.rand((B, H, W), device="cuda") * 100
    for _ in range(args.reps):
        net.infer(f, d2_sub=d2, raw=False)
    torch.cuda.synchronize()
    net.close()
    return f"net images={B} reps={args.reps}"


def run_train(nat, torch, args):
    B, H, W = args.pairs, 480, 640
    rng = np.random.default_rng(1)
    x = np.zeros((B, H, W, 8), np.float32)
    x[..., :4] = rng.uniform(0, 1, (B, H, W, 4)).astype(np.float32)
    f = torch.from_numpy((x.view(np.uint32) >> 16).astype(np.uint16)).cuda().view(torch.int16)
    t = torch.from_numpy(rng.uniform(-1.5, 1.5, (B, H, W)).astype(np.float32)).cuda()
    v = torch.from_numpy((rng.random((B, H, W)) < 0.85).astype(np.uint8)).cuda()
    net = nat.Net(B * H * W, seed=1)
    net.train_step(f, t, v, 1e-3)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.reps):
        net.train_step(f, t, v, 1e-3)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.reps * 1000
    net.close()
    return f"train batch={B} {W}x{H} steps={args.reps}: {ms:.3f} ms/step"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("workload", choices=("pair", "batch", "net", "train"))
    ap.add_argument("--paths", type=int, default=8)
    ap.add_argument("--pairs", type=int, default=64)
    ap.add_argument("--reps", type=int, default=4)
    ap.add_argument("--forms", choices=("both", "learned", "plain"), default="both",
                    help="batch: which forms to run (256 plain 8-path slots need ~250 GB)")
    args = ap.parse_args(argv)
    import torch
    import paper_2201_11924_amd.native as nat
    fn = {"pair": run_pair, "batch": run_batch, "net": run_net, "train": run_train}[args.workload]
    print(fn(nat, torch, args), flush=True)


if __name__ == "__main__":
    main()
