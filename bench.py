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

# algorithmic work of the aggregation pass per (pixel, disparity, path), the
# recurrence's own operations: min(L(d-1), L(d+1)), +P1, min with L(d), min with
# m + P2, +C, -m, the share of the path minimum m, and the accumulation into the
# summed cost (the cost itself, XOR + popcount, is not counted)
AGG_OPS_PER_PDR = 8
# MI355X: 256 CUs x 64 32-bit VALU lanes per clock x 2.4 GHz; packed 16-bit
# instructions do two lane-operations each
VALU_PEAK_OPS = 256 * 64 * 2.4e9
VALU_PEAK_OPS_PACKED16 = 2 * VALU_PEAK_OPS
HBM_PEAK = 8.0e12
# the machine's CPU share for one GPU (worker pools are sized to it)
HOST_POOL_MAX = 16


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the learned-form and batch legs")
    ap.add_argument("--batch-pairs", type=int, default=256)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--calibration-copy-mb", type=int, default=0,
                    help="after the timed steps, copy a buffer of this many MiB three times (a plain copy "
                         "kernel of known size, the reference for hardware traffic counters)")
    ap.add_argument("--no-paper-shape", action="store_true",
                    help="skip the leg at the paper's own timing shape (960x540, 4 paths, D in 64..256)")
    ap.add_argument("--cpu-sample-rows", type=int, default=720,
                    help="rows of the 1280x720 pair the oracle times (full pair = 720)")
    return ap.parse_args()


AGG_SOURCES = ("aggregate_impl.h", "aggregate.hip", "agg_dpl8.hip")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "aggregate_queue_1280x720_d128_8path_traffic.md")


def aggregation_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in AGG_SOURCES:
        with open(os.path.join(ROOT, "paper_2201_11924_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per aggregation launch from the committed counter summary, or None
    when the aggregation sources have changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return None
    fields = {}
    with open(TRAFFIC_PROFILE) as f:
        for line in f:
            if ":" in line and line.startswith("- `"):
                k, v = line[3:].split("`", 1)[0], line.split(":", 1)[1].strip()
                fields[k] = v
    if fields.get("source_sha256") != aggregation_source_hash():
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _oracle_pair(job):
    """One pair through the oracle (noise .. depth); returns the seconds it took."""
    from oracle import oracle as orc
    params, raw = job
    t0 = time.perf_counter()
    L = orc.ir_noise(raw[0], raw[2], raw[3])
    R = orc.ir_noise(raw[1], raw[4], raw[5])
    orc.sgm(params, L, R)
    return time.perf_counter() - t0


def _load_oracle(_):
    from oracle import oracle as orc
    orc.lib()


def _pool_rate(jobs, workers):
    """Pairs per second of the oracle over `jobs` on `workers` host processes
    (dynamic scheduling, one pair per task); wall clock of the whole map."""
    from multiprocessing import get_context
    with get_context("spawn").Pool(workers) as pool:
        pool.map(_load_oracle, range(workers), chunksize=1)  # start-up and oracle load, untimed
        t0 = time.perf_counter()
        pool.map(_oracle_pair, jobs, chunksize=1)
        wall = time.perf_counter() - t0
    return len(jobs) / wall, wall


def cpu_baseline(params, left, right, rows, workers):
    """The oracle as it stands on the host: single-threaded legs on one pair of
    the 320x240 and 1280x720 workloads, and all-cores legs (one process per core,
    pairs spread over them) on the uneven 64-pair batch and on 16 sensor pairs."""
    from oracle import oracle as orc
    from synth import CONFIGS, pair_seed
    from synth.stereo import sensor_like
    orc.build(force=False)
    legs = {}
    p = dict(params, height=rows)
    t0 = time.perf_counter()
    orc.sgm(p, np.ascontiguousarray(left[:rows]), np.ascontiguousarray(right[:rows]))
    dt = time.perf_counter() - t0
    legs["pair_1280x720_d128_1thread"] = {"pairs_s": round(rows / params["height"] / dt, 5), "cores": 1,
                                           "sample": f"{rows} of 720 rows, census..depth, {dt:.2f} s"}
    c0 = CONFIGS["pair_320x240_d64"]
    raw0 = _pool_generate([(c0["spec"], pair_seed(0, 0))], 1)[0]
    ts = sorted(_oracle_pair((c0["params"], raw0)) for _ in range(5))
    legs["pair_320x240_d64_1thread"] = {"pairs_s": round(1.0 / ts[2], 4), "cores": 1,
                                         "sample": "one pair, noise..depth, median of 5 runs"}
    shapes = [(320, 240, 64), (640, 480, 96), (848, 480, 128), (1280, 720, 128)]
    specs, plist = [], []
    for si, (w, h, d) in enumerate(shapes):
        c = sensor_like(w, h, d)
        for i in range(16):
            specs.append((c["spec"], pair_seed(2, 16 * si + i)))
            plist.append(c["params"])
    raws = _pool_generate(specs, workers)
    rate, wall = _pool_rate(list(zip(plist, raws)), workers)
    work = sum(q["width"] * q["height"] * q["max_disp"] for q in plist)
    legs["batch_64_uneven_all_cores"] = {"pairs_s": round(rate, 4), "cores": workers, "wall_s": round(wall, 2),
                                         "mpix_disp_per_s": round(work / wall / 1e6, 2),
                                         "sample": "the whole 64-pair batch, noise..depth per pair"}
    c1 = CONFIGS["pair_1280x720_d128"]
    raws = _pool_generate([(c1["spec"], pair_seed(4, i)) for i in range(16)], workers)
    rate, wall = _pool_rate([(c1["params"], r) for r in raws], workers)
    legs["sensor_16_pairs_all_cores"] = {"pairs_s": round(rate, 4), "cores": workers, "wall_s": round(wall, 2),
                                         "sample": "16 of the 256 sensor pairs (32 cameras x 8 steps), plain "
                                                   "8-path, noise..depth per pair"}
    return {"value": legs["sensor_16_pairs_all_cores"]["pairs_s"], "unit": "pairs/s", "cores": workers,
            "host_cores": os.cpu_count(), "kind": "oracle",
            "sample": f"16 1280x720 D=128 8-path pairs (the headline shape), one oracle process per core on "
                      f"{workers} of the host's {os.cpu_count()} cores, noise..depth, wall clock",
            "legs": legs}


def _pool_generate(spec_seeds, workers):
    from paper_2201_11924_amd.train import generate
    return generate(spec_seeds, workers)


def generate_batch_inputs(args):
    """Host-side pair generation for the batch legs, in worker processes started
    before this process touches the GPU."""
    from synth import CONFIGS, pair_seed
    from synth.stereo import sensor_like
    cfg = CONFIGS["pair_1280x720_d128"]
    sensor = _pool_generate([(cfg["spec"], pair_seed(4, i)) for i in range(args.batch_pairs)], args.workers)
    shapes = [(320, 240, 64), (640, 480, 96), (848, 480, 128), (1280, 720, 128)]
    specs, plist = [], []
    for si, (w, h, d) in enumerate(shapes):
        c = sensor_like(w, h, d)
        for i in range(16):
            specs.append((c["spec"], pair_seed(2, 16 * si + i)))
            plist.append(c["params"])
    uneven = _pool_generate(specs, args.workers)
    return sensor, (uneven, plist)


def pairs_in_flight_leg(nat, params, raw, H, W, n_pairs=300):
    """The headline step (IR noise on both images, then the plain 8-path path) over a
    run of pairs handed out in turn to k handles, each on a stream of its own, so that
    up to k pairs are in flight: one pair's selection (bound by HBM) can then overlap
    another's aggregation (bound by the vector ALUs).  Every pair is still computed
    whole; k = 1 is the headline's sequential step."""
    import torch
    c2, g2, n2 = raw
    res = {}
    for k in (1, 2, 3):
        hs = [nat.SimSense(params) for _ in range(k)]
        sts = [torch.cuda.Stream() for _ in range(k)]
        bufs = [dict(LR=torch.empty_like(c2),
                     out=[torch.empty((H, W), dtype=torch.float32, device=c2.device) for _ in range(2)] +
                         [torch.empty((H, W), dtype=torch.uint8, device=c2.device)]) for _ in range(k)]

        def run(n):
            for i in range(n):
                j = i % k
                st, b = sts[j], bufs[j]
                nat.ir_noise(c2, g2, n2, out=b["LR"], stream=st)
                hs[j].compute(b["LR"][0], b["LR"][1], *b["out"], stream=st)

        run(6 * k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(n_pairs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[f"{k}_in_flight"] = {"pairs_s": round(n_pairs / dt, 1), "handles": k, "pairs": n_pairs}
        for h in hs:
            h.close()
    res["note"] = ("the headline step over a run of pairs dealt in turn to k handles on k streams; "
                   "wall clock over the run, inputs resident")
    return res


def learned_and_batch_legs(nat, args, out, inputs):
    """The learned 2-path+net form against plain 8-path, and uneven batches."""
    import torch
    from paper_2201_11924_amd.train import load_checkpoint, metrics
    from synth import CONFIGS, pair_seed
    from synth.stereo import sensor_like
    cfg = CONFIGS["pair_1280x720_d128"]
    params8 = cfg["params"]
    params2 = dict(params8, num_paths=2)
    W, H, D = params8["width"], params8["height"], params8["max_disp"]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    ck = os.path.join(ROOT, "paper_2201_11924_amd", "weights", "surrogate_640x480_d128.ckpt")
    chunk = 16
    net = nat.Net(chunk * W * H, seed=0)
    trained = os.path.exists(ck)
    if trained:
        load_checkpoint(ck, net)

    # single pair, learned form
    raw = inputs[0][0]
    L = nat.ir_noise(t(raw[0]), t(raw[2]), t(raw[3]))
    R = nat.ir_noise(t(raw[1]), t(raw[4]), t(raw[5]))
    ss2 = nat.SimSense(params2)
    for _ in range(10):
        nat.learned_compute(ss2, net, L, R)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = max(20, args.steps // 4)
    for _ in range(reps):
        nat.learned_compute(ss2, net, L, R)
    e1.record()
    torch.cuda.synchronize()
    ms_l = e0.elapsed_time(e1) / reps
    ss2.close()
    res = {"single_pair_2path_net": {"pairs_s": round(1000.0 / ms_l, 2), "ms": round(ms_l, 4)}}

    # 256 pairs (32 cameras x 8 steps) of the sensor workload
    npairs = args.batch_pairs
    raws = inputs[0]
    Ls, Rs = [], []
    for r in raws:
        Ls.append(nat.ir_noise(t(r[0]), t(r[2]), t(r[3])))
        Rs.append(nat.ir_noise(t(r[1]), t(r[4]), t(r[5])))
    del raws
    torch.cuda.synchronize()
    # plain 8-path in graph launches of 64 pairs
    g8 = min(64, npairs)
    b8 = nat.Batch([params8] * g8)
    outs8 = [b8.outputs() for _ in range(0, npairs, g8)]
    tune8, _ = b8.autotune(Ls[:g8], Rs[:g8], outs8[0], reps=2)  # launch shape, as for the learned form
    for i in range(0, npairs, g8):
        b8.compute(Ls[i:i + g8], Rs[i:i + g8], outs8[i // g8])
    torch.cuda.synchronize()
    e0.record()
    for i in range(0, npairs, g8):
        b8.compute(Ls[i:i + g8], Rs[i:i + g8], outs8[i // g8])
    e1.record()
    torch.cuda.synchronize()
    ms8 = e0.elapsed_time(e1)
    b8.close()
    # learned form, every pair in one graph launch (no fallback)
    b2 = nat.Batch([params2] * npairs)
    outs2 = b2.outputs()
    tune2, _ = b2.autotune(Ls, Rs, outs2, reps=2)  # launch shape for the 2-path matching
    unc = torch.zeros(npairs, dtype=torch.int32, device="cuda")
    tau = 0.5
    b2.learned_compute(net, Ls, Rs, outs2, tau, unc)
    torch.cuda.synchronize()
    e0.record()
    b2.learned_compute(net, Ls, Rs, outs2, tau, unc)
    e1.record()
    torch.cuda.synchronize()
    ms2 = e0.elapsed_time(e1)
    d8 = [outs8[i // g8][i % g8]["disp"].cpu().numpy() for i in range(npairs)]
    q = [metrics(outs2[i]["disp"].cpu().numpy(), d8[i]) for i in range(npairs)]
    qm = {k: round(float(np.mean([m[k] for m in q])), 5) for k in q[0]}
    # the learned form with plain 8-path SGM as its fallback, run for real: pairs
    # whose share of uncertain logits (|logit| < tau) passes the limit are
    # recomputed by an 8-path handle over their own outputs; the limit is the
    # 90th percentile of the shares of the untimed pass above
    frac_unsure = unc.cpu().numpy() / float(W * H)
    limit = float(np.quantile(frac_unsure, 0.9))
    plain = nat.SimSense(params8)
    b2.learned_fallback(net, plain, Ls, Rs, outs2, tau, unc, nat.FALLBACK_THRESHOLD, limit)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    fb = b2.learned_fallback(net, plain, Ls, Rs, outs2, tau, unc, nat.FALLBACK_THRESHOLD, limit)
    e1.record()
    torch.cuda.synchronize()
    ms_fb = max(e0.elapsed_time(e1), (time.perf_counter() - t0) * 1000.0)  # (the call waits once on the host)
    plain.close()
    qf = [metrics(outs2[i]["disp"].cpu().numpy(), d8[i]) for i in range(npairs)]
    qfm = {k: round(float(np.mean([m[k] for m in qf])), 5) for k in qf[0]}
    pairs8 = npairs / (ms8 / 1000.0)
    pairs2 = npairs / (ms2 / 1000.0)
    pairs_fb = npairs / (ms_fb / 1000.0)
    res["batch_256_sensor"] = {
        "pairs": npairs, "plain_8path_pairs_s": round(pairs8, 2), "learned_2path_net_pairs_s": round(pairs2, 2),
        "speedup": round(pairs2 / pairs8, 3), "plain_graph_launches": (npairs + g8 - 1) // g8,
        "learned_graph_launches": 1, "net_trained": trained, "plain_tuning": tune8, "learned_tuning": tune2,
        "quality_vs_8path": qm,
        "with_fallback": {"tau": tau, "limit_uncertain_share": round(limit, 5), "rate": round(sum(fb) / npairs, 4),
                          "pairs_s": round(pairs_fb, 2), "speedup": round(pairs_fb / pairs8, 3),
                          "quality_vs_8path": qfm,
                          "how": "simsense_batch_learned_fallback: learned graph, per-pair counts to the host, "
                                 "plain 8-path handle on the flagged pairs; timed as one call"}}
    b2.close()
    net.close()
    del Ls, Rs, outs2, outs8
    torch.cuda.empty_cache()

    # 64 pairs of uneven sizes and disparity ranges in one graph launch, autotuned
    raws, plist = inputs[1]
    Ls = [nat.ir_noise(t(r[0]), t(r[2]), t(r[3])) for r in raws]
    Rs = [nat.ir_noise(t(r[1]), t(r[4]), t(r[5])) for r in raws]
    del raws
    bu = nat.Batch(plist)
    outs = bu.outputs()
    best, cand = bu.autotune(Ls, Rs, outs, reps=3)
    bu.compute(Ls, Rs, outs)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        bu.compute(Ls, Rs, outs)
    e1.record()
    torch.cuda.synchronize()
    msu = e0.elapsed_time(e1) / 5
    work = sum(p["width"] * p["height"] * p["max_disp"] for p in plist)
    res["batch_64_uneven"] = {"pairs_s": round(64 / (msu / 1000.0), 2), "ms_per_launch": round(msu, 3),
                              "mpix_disp_per_s": round(work / (msu / 1000.0) / 1e6, 1), "tuning": best,
                              "autotune_ms": [round(m, 3) for m in cand]}
    bu.close()
    out["learned_and_batches"] = res


# Sec. VI-D, Table II: SGM frames/s of the paper's implementation at 960x540 with
# 4 paths on an NVIDIA RTX 4090 (another GPU; quoted as context only)
PAPER_TABLE2_SGM_FPS = {64: 414.51, 96: 326.79, 128: 281.26, 256: 147.13}
PAPER_TABLE2_SGBM_FPS = {64: 342.24, 96: 268.98, 128: 232.49, 256: 128.56}
SGBM_BLOCK = 3  # the paper gives no block size; penalties scale with the block area


def paper_shape_leg(nat, reps=100):
    """Plain SGM at the shape the paper times: 960x540, 4 paths, D = 64/96/128/256."""
    import torch
    from synth import make_pair, pair_seed
    from synth.stereo import sensor_like
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    res, res_b = {}, {}
    for i, D in enumerate(sorted(PAPER_TABLE2_SGM_FPS)):
        cfg = sensor_like(960, 540, D)
        pr = make_pair(cfg["spec"], pair_seed(5, i))
        L = nat.ir_noise(t(pr.left), t(pr.gamma_l), t(pr.n_l))
        R = nat.ir_noise(t(pr.right), t(pr.gamma_r), t(pr.n_r))
        depth = torch.empty((540, 960), dtype=torch.float32, device="cuda")
        a = SGBM_BLOCK * SGBM_BLOCK
        sgm = dict(cfg["params"], num_paths=4)
        sgbm = dict(sgm, block_w=SGBM_BLOCK, block_h=SGBM_BLOCK, p1=sgm["p1"] * a, p2=sgm["p2"] * a)
        for params, out, paper in ((sgm, res, PAPER_TABLE2_SGM_FPS), (sgbm, res_b, PAPER_TABLE2_SGBM_FPS)):
            ss = nat.SimSense(params)
            for _ in range(10):
                ss.compute(L, R, depth)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                ss.compute(L, R, depth)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            ss.close()
            fps = 1000.0 / ms
            out[f"D{D}"] = {"fps": round(fps, 1), "ms": round(ms, 4),
                            "mpix_disp_per_s": round(960 * 540 * D * fps / 1e6, 1), "paper_fps_rtx4090": paper[D]}
            if params is sgm:
                # the paper's whole timed chain: rectify both raw images, match, register
                # the depth into a 1920x1080 RGB camera
                ys, xs = torch.meshgrid(torch.arange(540, device="cuda", dtype=torch.float32),
                                        torch.arange(960, device="cuda", dtype=torch.float32), indexing="ij")
                mx, my = (xs + 0.37).contiguous(), (ys - 0.21).contiguous()
                ir = (params["focal_px"] * 0.75, params["focal_px"] * 0.75, 479.5, 269.5)
                rgb = (1380.0, 1380.0, 959.5, 539.5)
                rt = [1, 0, 0, 0, 1, 0, 0, 0, 1, -0.015, 0.0, 0.0]
                ss = nat.SimSense(params)

                def chain():
                    Lr = nat.rectify(L, mx, my)
                    Rr = nat.rectify(R, mx, my)
                    ss.compute(Lr, Rr, depth)
                    return nat.register_depth(depth, ir, rt, rgb, 1920, 1080)
                for _ in range(10):
                    chain()
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    chain()
                e1.record()
                torch.cuda.synchronize()
                msc = e0.elapsed_time(e1) / reps
                ss.close()
                out[f"D{D}"]["fps_rectify_match_register_1920x1080"] = round(1000.0 / msc, 1)
    return {"shape": "960x540, 4 paths, census 7x9 CS, depth output at 960x540 (the paper's 1920x1080 "
                     "registration is not part of this path)", "by_max_disp": res,
            "sgbm": {"block": f"{SGBM_BLOCK}x{SGBM_BLOCK}, P1/P2 x {SGBM_BLOCK * SGBM_BLOCK}", "by_max_disp": res_b}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    inputs = None if args.no_batch else generate_batch_inputs(args)

    import torch
    import paper_2201_11924_amd.native as nat
    from synth import CONFIGS, make_pair, pair_seed

    cfg = CONFIGS["pair_1280x720_d128"]
    params = cfg["params"]
    W, H, D, P = params["width"], params["height"], params["max_disp"], params["num_paths"]
    pair = make_pair(cfg["spec"], pair_seed(1, 0))
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    # the two images, their draws and the noisy pair stacked, so that the noise model
    # of both images is one elementwise call over 2 x H x W pixels
    c2 = t(np.stack([pair.left, pair.right]))
    g2 = t(np.stack([pair.gamma_l, pair.gamma_r]))
    n2 = t(np.stack([pair.n_l, pair.n_r]))
    LR = torch.empty_like(c2)
    L, R = LR[0], LR[1]
    depth = torch.empty((H, W), dtype=torch.float32, device=dev)
    disp = torch.empty_like(depth)
    flags = torch.empty((H, W), dtype=torch.uint8, device=dev)
    ss = nat.SimSense(params)

    def step():
        nat.ir_noise(c2, g2, n2, out=LR)
        ss.compute(L, R, depth, disp, flags)

    for _ in range(args.warmup):
        step()
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
    ms_step = ms_total / args.steps
    # per-pass device times: the same steps again, with the library's per-pass
    # HIP events recorded on the launch stream around each pass
    ss.profile(True)
    ss.profile_read()
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    end.record()
    torch.cuda.synchronize()
    ms_step_profiled = start.elapsed_time(end) / args.steps
    calls, pass_ms = ss.profile_read()
    ss.profile(False)
    pairs_s = 1000.0 / ms_step
    vol = W * H * D

    agg_s = pass_ms["aggregate"] / calls / 1000.0
    agg_ops = AGG_OPS_PER_PDR * P * vol
    achieved = agg_ops / agg_s
    kernel = "aggregate_queue_kernel" if ss.get_tuning()["blocks_per_cu"] > 0 else "aggregate_kernel"
    # the kernel's path arithmetic runs in 32-bit lanes, so its peak is the
    # 32-bit one; the packed 16-bit peak (what a u16 form could reach) is beside it
    roofline = {"kernel": kernel, "bound": "alu", "achieved": round(achieved / 1e12, 3),
                "peak": round(VALU_PEAK_OPS / 1e12, 3), "unit": "Tops/s", "frac": round(achieved / VALU_PEAK_OPS, 4),
                "traffic": measured_traffic(),
                "peak_packed_u16": round(VALU_PEAK_OPS_PACKED16 / 1e12, 3),
                "frac_packed_u16": round(achieved / VALU_PEAK_OPS_PACKED16, 4),
                "ops_per_pixel_disp_path": AGG_OPS_PER_PDR,
                "ops_per_launch": agg_ops, "avg_launch_us": round(agg_s * 1e6, 2),
                "timed_by": "library per-pass HIP events on the launch stream, second timed loop of the same steps"}
    # floors of the whole step: with 8 paths the summed costs cannot stay on
    # chip, so at least one uint16 write and read of W*H*D values, plus the two
    # images in and depth, disparity and flags out; and the aggregation's
    # operations at the VALU peak
    step_s = ms_step / 1000.0
    hbm_floor_bytes = 4 * vol + (2 + 4 + 4 + 1) * W * H
    floors = {"hbm_bytes": hbm_floor_bytes, "hbm_us": round(hbm_floor_bytes / HBM_PEAK * 1e6, 2),
              "valu_ops": agg_ops, "valu_us": round(agg_ops / VALU_PEAK_OPS * 1e6, 2),
              "step_us": round(step_s * 1e6, 2),
              "hbm_frac": round(hbm_floor_bytes / HBM_PEAK / step_s, 4),
              "valu_frac": round(agg_ops / VALU_PEAK_OPS / step_s, 4)}
    floors["roofline_fraction"] = max(floors["hbm_frac"], floors["valu_frac"])
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
        "ms_per_step_with_pass_events": round(ms_step_profiled, 5),
        "wall_s": round(wall, 3),
        "roofline": roofline,
        "step_floors": floors,
    }
    ss.close()
    if not args.no_paper_shape:
        # the same pair with the LR check against a full right-referenced run
        ssr = nat.SimSense(dict(params, lr_mode=1))
        for _ in range(5):
            ssr.compute(L, R, depth, disp, flags)
        start.record()
        for _ in range(50):
            ssr.compute(L, R, depth, disp, flags)
        end.record()
        torch.cuda.synchronize()
        msr = start.elapsed_time(end) / 50
        ssr.close()
        out["lr_full_right_run"] = {"pairs_s": round(1000.0 / msr, 2), "ms": round(msr, 4)}
        out["pairs_in_flight"] = pairs_in_flight_leg(nat, params, (c2, g2, n2), H, W)
    if args.calibration_copy_mb > 0:
        n = args.calibration_copy_mb << 20
        src = torch.empty(n, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = n
        del src, dst
    if not args.no_paper_shape:
        out["paper_shape_4path_960x540"] = paper_shape_leg(nat)
    if not args.no_batch:
        learned_and_batch_legs(nat, args, out, inputs)
        inputs = None
    if not args.no_cpu_baseline:
        from oracle import oracle as orc
        Lh = orc.ir_noise(pair.left, pair.gamma_l, pair.n_l)
        Rh = orc.ir_noise(pair.right, pair.gamma_r, pair.n_r)
        workers = max(1, min(HOST_POOL_MAX, os.cpu_count() or 1))
        out["cpu_baseline"] = cpu_baseline(params, Lh, Rh, args.cpu_sample_rows, workers)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
