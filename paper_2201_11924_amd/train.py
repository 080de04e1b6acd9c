"""Training and evaluation driver of the learned surrogate.

Pipeline per synthetic pair (all on the GPU through the C ABI): IR noise on both
images, plain 8-path SGM (the target: its sub-pixel disparity and validity),
2-path SGM with the net's features, then the training targets
(residual = d8_sub - d2_sub, validity of the 8-path result).  Training runs
Adam steps on batches of pairs; evaluation compares the learned form and the
plain 2-path form against 8-path SGM.

Checkpoints are a JSON header line followed by the raw little-endian fp32
parameter, first-moment and second-moment vectors.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from multiprocessing import get_context
from typing import Dict, List, Optional

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synth.stereo import sensor_like, make_pair, pair_seed  # noqa: E402


def _gen(args):
    spec, seed = args
    p = make_pair(spec, seed)
    return p.left, p.right, p.gamma_l, p.n_l, p.gamma_r, p.n_r


def generate(specs_seeds, workers: int = 8):
    """Host-side pair generation, in parallel (call before the GPU is initialised
    or with the spawn start method)."""
    if workers <= 1:
        return [_gen(a) for a in specs_seeds]
    with get_context("spawn").Pool(workers) as pool:
        return pool.map(_gen, specs_seeds, chunksize=4)


class PairRunner:
    """Runs 8-path and 2-path matching on noisy pairs of one size."""

    def __init__(self, nat, params: Dict):
        import torch
        self.torch = torch
        self.nat = nat
        self.p8 = dict(params, num_paths=8)
        self.p2 = dict(params, num_paths=2)
        self.ss8 = nat.SimSense(self.p8)
        self.ss2 = nat.SimSense(self.p2)
        self.H, self.W = params["height"], params["width"]

    def noisy(self, raw):
        t = lambda a: self.torch.from_numpy(np.ascontiguousarray(a)).cuda()
        left, right, gl, nl, gr, nr = raw
        return self.nat.ir_noise(t(left), t(gl), t(nl)), self.nat.ir_noise(t(right), t(gr), t(nr))

    def sample(self, raw):
        """features (int16 bits of bf16), t_res, t_valid, d2 outputs, d8 outputs."""
        L, R = self.noisy(raw)
        o8 = self.ss8.compute_all(L, R)
        o2 = self.ss2.compute_all(L, R, features=True)
        t_res, t_valid = self.nat.net_targets(o8["disp_sub"], o8["flags"], o2["disp_sub"])
        return dict(L=L, R=R, features=o2["features"], t_res=t_res, t_valid=t_valid, d8=o8["disp"],
                    f8=o8["flags"], d2=o2["disp"], f2=o2["flags"])

    def close(self):
        self.ss8.close()
        self.ss2.close()


def metrics(disp: np.ndarray, d8: np.ndarray) -> Dict[str, float]:
    """Quality against 8-path SGM: share of 8-path-valid pixels more than 1 px off
    (invalid counts as off), mask agreement, and the share of 8-path-valid pixels
    the form marks valid."""
    v8 = d8 > 0
    v = disp > 0
    off = v8 & (~v | (np.abs(disp - d8) > 1.0))
    return dict(bad1=float(off.sum() / max(v8.sum(), 1)),
                bad1_where_valid=float((v8 & v & (np.abs(disp - d8) > 1.0)).sum() / max((v8 & v).sum(), 1)),
                mask_agree=float((v == v8).mean()), recall=float((v & v8).sum() / max(v8.sum(), 1)),
                valid=float(v.mean()))


def save_checkpoint(path: str, net, meta: Optional[dict] = None) -> None:
    p, m, v, step = net.get_state()
    head = dict(meta or {}, format="simsense-net-v1", num_params=int(p.size), step=int(step),
                layout="params,m,v as little-endian float32")
    with open(path, "wb") as f:
        f.write((json.dumps(head) + "\n").encode())
        for a in (p, m, v):
            f.write(np.ascontiguousarray(a, "<f4").tobytes())


def load_checkpoint(path: str, net) -> dict:
    with open(path, "rb") as f:
        head = json.loads(f.readline().decode())
        n = int(head["num_params"])
        arrs = [np.frombuffer(f.read(4 * n), dtype="<f4").astype(np.float32) for _ in range(3)]
    net.set_state(arrs[0], arrs[1], arrs[2], int(head["step"]))
    return head


def build_dataset(runner: PairRunner, raws) -> Dict:
    """Training tensors on the GPU from raw pairs (a list, or an iterable of lists
    generated chunk by chunk so that the raw images of every pair need not be
    held on the host at once)."""
    import torch
    feats, tres, tval = [], [], []
    chunks = [raws] if isinstance(raws, list) else raws
    for chunk in chunks:
        for raw in chunk:
            s = runner.sample(raw)
            feats.append(s["features"])
            tres.append(s["t_res"])
            tval.append(s["t_valid"])
        torch.cuda.synchronize()
    return dict(features=torch.stack(feats), t_res=torch.stack(tres), t_valid=torch.stack(tval))


def lr_at(it: int, steps: int, lr: float, schedule: str, min_lr: float) -> float:
    """Learning rate of step `it`: constant, or cosine decay from lr to min_lr."""
    if schedule == "cosine" and steps > 1:
        return min_lr + 0.5 * (lr - min_lr) * (1.0 + math.cos(math.pi * it / (steps - 1)))
    return lr


def train(net, data: Dict, steps: int, batch: int, lr: float, seed: int = 0, log=None, schedule: str = "constant",
          min_lr: float = 0.0) -> List[float]:
    import torch
    n = data["features"].shape[0]
    rng = np.random.default_rng(seed)
    order = rng.permutation(n)
    pos = 0
    losses = []
    for it in range(steps):
        if pos + batch > n:
            order = rng.permutation(n)
            pos = 0
        idx = torch.from_numpy(order[pos:pos + batch]).cuda()
        pos += batch
        f = data["features"].index_select(0, idx).contiguous()
        t = data["t_res"].index_select(0, idx).contiguous()
        v = data["t_valid"].index_select(0, idx).contiguous()
        loss = net.train_step(f, t, v, lr_at(it, steps, lr, schedule, min_lr))
        if log is not None and (it % 25 == 0 or it == steps - 1):
            lv = loss.cpu().numpy()
            losses.append(float(lv[0]))
            log(json.dumps({"step": it, "loss": float(lv[0]), "l1": float(lv[1]), "bce": float(lv[2])}))
    return losses


def evaluate(nat, runner: PairRunner, net, raws: List) -> Dict[str, float]:
    import torch
    acc = {"net": [], "two_path": []}
    for raw in raws:
        s = runner.sample(raw)
        out = nat.learned_compute(runner.ss2, net, s["L"], s["R"])
        torch.cuda.synchronize()
        d8 = s["d8"].cpu().numpy()
        acc["net"].append(metrics(out["disp"].cpu().numpy(), d8))
        acc["two_path"].append(metrics(s["d2"].cpu().numpy(), d8))
    return {form: {k: float(np.mean([m[k] for m in ms])) for k in ms[0]} for form, ms in acc.items()}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--eval-pairs", type=int, default=16)
    ap.add_argument("--width", type=int, default=640)
    ap.add_argument("--height", type=int, default=480)
    ap.add_argument("--max-disp", type=int, default=128)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--schedule", choices=("constant", "cosine"), default="constant")
    ap.add_argument("--min-lr", type=float, default=1e-5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--out", default=None, help="checkpoint path")
    ap.add_argument("--resume", default=None)
    ap.add_argument("--chunk", type=int, default=0,
                    help="generate and convert the training pairs this many at a time (0: all at once)")
    ap.add_argument("--seed-offset", type=int, default=0,
                    help="first pair index of the training seeds (pair_seed(3, offset + i))")
    args = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)

    cfg = sensor_like(args.width, args.height, args.max_disp)
    t0 = time.time()
    specs = [(cfg["spec"], pair_seed(3, args.seed_offset + i)) for i in range(args.pairs)]
    train_raw = generate(specs, args.workers) if args.chunk <= 0 else None
    eval_raw = generate([(cfg["spec"], pair_seed(3, 1_000 + i) + 500_000) for i in range(args.eval_pairs)],
                        args.workers)
    log(json.dumps({"generated": len(eval_raw) + (len(train_raw) if train_raw else 0), "s": round(time.time() - t0, 1)}))

    import torch
    import paper_2201_11924_amd.native as nat
    runner = PairRunner(nat, cfg["params"])
    t0 = time.time()
    if train_raw is None:
        # each chunk is generated by spawned workers when the previous one is converted
        chunks = (generate(specs[i:i + args.chunk], args.workers) for i in range(0, len(specs), args.chunk))
        data = build_dataset(runner, chunks)
    else:
        data = build_dataset(runner, train_raw)
    del train_raw
    log(json.dumps({"dataset_pairs": int(data["features"].shape[0]), "s": round(time.time() - t0, 1),
                    "valid8_share": float(data["t_valid"].float().mean())}))
    net = nat.Net(args.batch * args.width * args.height, seed=args.seed)
    if args.resume:
        load_checkpoint(args.resume, net)
    before = evaluate(nat, runner, net, eval_raw)
    t0 = time.time()
    losses = train(net, data, args.steps, args.batch, args.lr, args.seed, log, args.schedule, args.min_lr)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    after = evaluate(nat, runner, net, eval_raw)
    res = {"train_steps": args.steps, "batch": args.batch, "train_s": round(train_s, 2),
           "steps_per_s": round(args.steps / train_s, 2), "loss_first": losses[0], "loss_last": losses[-1],
           "eval_untrained": before, "eval_trained": after}
    log(json.dumps(res))
    if args.out:
        save_checkpoint(args.out, net, dict(pairs=args.pairs, steps=args.steps, batch=args.batch, lr=args.lr,
                                            schedule=args.schedule, min_lr=args.min_lr, resumed_from=args.resume,
                                            width=args.width, height=args.height, max_disp=args.max_disp))
    runner.close()
    net.close()
    return res


if __name__ == "__main__":
    main()
