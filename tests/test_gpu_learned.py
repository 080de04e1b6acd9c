"""The learned 2-path+net form at the sensor shape: its fallback to plain 8-path
SGM, what the trained net gains over 2-path alone on held-out pairs, and the
1280x720 batch and fused-inference cases.

Every comparison target is either the oracle or a single-pair path that the
oracle checks elsewhere (plain SGM at 1280x720 in test_gpu_parity.py, the fused
net against the layered forward in test_gpu_net.py)."""
import os

import numpy as np
import pytest

from synth import make_pair, pair_seed
from synth.stereo import sensor_like

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CKPT = os.path.join(ROOT, "paper_2201_11924_amd", "weights", "surrogate_640x480_d128.ckpt")
HELD_OUT = 6  # workload index of the held-out pairs: never used for training (index 3) or benchmarking


@pytest.fixture(scope="module")
def nat():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_11924_amd.native as n
    return n


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def noisy_pairs(orc, cfg, seeds):
    Ls, Rs = [], []
    for s in seeds:
        pr = make_pair(cfg["spec"], s)
        Ls.append(dev(orc.ir_noise(pr.left, pr.gamma_l, pr.n_l)))
        Rs.append(dev(orc.ir_noise(pr.right, pr.gamma_r, pr.n_r)))
    return Ls, Rs


def trained_net(nat, max_pixels):
    from paper_2201_11924_amd.train import load_checkpoint
    net = nat.Net(max_pixels, seed=0)
    load_checkpoint(CKPT, net)
    return net


def random_net(nat, max_pixels, seed):
    from oracle import net_oracle as no
    rng = np.random.default_rng(seed)
    params = [(w, rng.uniform(-0.05, 0.05, b.shape)) for w, b in no.init_params(seed)]
    net = nat.Net(max_pixels, seed=0)
    net.set_state(no.flatten(params))
    return net


def host(o):
    return {k: v.cpu().numpy() for k, v in o.items()}


def test_fallback_modes(orc, nat):
    """NEVER leaves the learned result, ALWAYS gives plain 8-path SGM for every pair,
    THRESHOLD recomputes exactly the pairs whose uncertain-pixel count exceeds the
    limit; every output equals its single-path result bit for bit."""
    import torch
    W, H, D = 200, 120, 64
    cfg = sensor_like(W, H, D)
    p2 = dict(cfg["params"], num_paths=2)
    p8 = dict(cfg["params"], num_paths=8)
    n = 5
    Ls, Rs = noisy_pairs(orc, cfg, [pair_seed(HELD_OUT, 100 + i) for i in range(n)])
    net = random_net(nat, W * H, 21)
    ss2 = nat.SimSense(p2)
    ss8 = nat.SimSense(p8)
    learned = [host(nat.learned_compute(ss2, net, l, r)) for l, r in zip(Ls, Rs)]
    plain = [host(dict(zip(("depth", "disp", "flags"), ss8(l, r)))) for l, r in zip(Ls, Rs)]
    torch.cuda.synchronize()
    b = nat.Batch([p2] * n)
    outs = b.outputs()
    unc = torch.zeros(n, dtype=torch.int32, device="cuda")
    tau = 0.5

    def check(fb, label):
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            want = plain[i] if fb[i] else learned[i]
            for k in ("depth", "disp", "flags"):
                assert np.array_equal(o[k].cpu().numpy(), want[k]), (label, i, k)

    fb = b.learned_fallback(net, None, Ls, Rs, outs, tau, unc, nat.FALLBACK_NEVER)
    assert fb == [0] * n
    check(fb, "never")
    counts = unc.cpu().numpy().astype(np.int64)
    fb = b.learned_fallback(net, ss8, Ls, Rs, outs, tau, unc, nat.FALLBACK_ALWAYS)
    assert fb == [1] * n
    check(fb, "always")
    # a limit between two of the observed counts: some pairs fall back, some do not
    srt = np.sort(counts)
    assert srt[0] < srt[-1], counts
    k = int(np.searchsorted(srt, srt[-1]) - 1)
    frac = (srt[k] + 0.5) / (W * H)
    fb = b.learned_fallback(net, ss8, Ls, Rs, outs, tau, unc, nat.FALLBACK_THRESHOLD, frac)
    assert fb == [int(c > frac * W * H) for c in counts]
    assert 0 < sum(fb) < n
    check(fb, "threshold")
    # argument checks
    with pytest.raises(nat.SimSenseError):
        b.learned_fallback(net, ss8, Ls, Rs, outs, tau, unc, 7)
    with pytest.raises(nat.SimSenseError):
        b.learned_fallback(net, None, Ls, Rs, outs, tau, unc, nat.FALLBACK_ALWAYS)
    wrong = nat.SimSense(dict(p8, max_disp=32))
    with pytest.raises(nat.SimSenseError):
        b.learned_fallback(net, wrong, Ls, Rs, outs, tau, unc, nat.FALLBACK_ALWAYS)
    for x in (b, ss2, ss8, wrong, net):
        x.close()


def test_trained_net_beats_two_path_alone_on_held_out_pairs(orc, nat):
    """What the trained net gains: on held-out sensor pairs (1280x720, D=128, seeds
    never used in training), the share of 8-path-valid pixels that are more than
    1 px off or dropped (bad1) is lower for 2-path+net than for 2-path SGM with its
    own uniqueness/LR masks (measured: 2.56% -> 1.59% on these four pairs), and more
    of the 8-path-valid pixels are kept (97.9% -> 99.2%)."""
    import torch
    from paper_2201_11924_amd.train import metrics
    cfg = sensor_like(1280, 720, 128)
    p2 = dict(cfg["params"], num_paths=2)
    p8 = dict(cfg["params"], num_paths=8)
    Ls, Rs = noisy_pairs(orc, cfg, [pair_seed(HELD_OUT, i) for i in range(4)])
    net = trained_net(nat, 1280 * 720)
    ss2, ss8 = nat.SimSense(p2), nat.SimSense(p8)
    m_net, m_two = [], []
    for l, r in zip(Ls, Rs):
        d8 = ss8(l, r)[1].cpu().numpy()
        d2 = ss2(l, r)[1].cpu().numpy()
        dn = nat.learned_compute(ss2, net, l, r)["disp"].cpu().numpy()
        m_net.append(metrics(dn, d8))
        m_two.append(metrics(d2, d8))
    mean = lambda ms, k: float(np.mean([m[k] for m in ms]))
    print(f"held-out bad1: 2-path {mean(m_two, 'bad1'):.4f}, 2-path+net {mean(m_net, 'bad1'):.4f}; "
          f"recall 2-path {mean(m_two, 'recall'):.4f}, 2-path+net {mean(m_net, 'recall'):.4f}")
    assert mean(m_net, "bad1") < 0.8 * mean(m_two, "bad1")
    assert mean(m_net, "recall") > mean(m_two, "recall")
    assert mean(m_net, "mask_agree") > mean(m_two, "mask_agree")
    for x in (ss2, ss8, net):
        x.close()


def test_learned_batch_at_sensor_shape_equals_single_pairs(orc, nat):
    """The learned batch at 1280x720, D=128 (the 256-pair workload's shape; 720 rows
    span many row segments of the fused kernel) equals the single-pair learned path."""
    import torch
    cfg = sensor_like(1280, 720, 128)
    p2 = dict(cfg["params"], num_paths=2)
    n = 3
    Ls, Rs = noisy_pairs(orc, cfg, [pair_seed(HELD_OUT, 200 + i) for i in range(n)])
    net = trained_net(nat, 1280 * 720)
    ss2 = nat.SimSense(p2)
    singles = [host(nat.learned_compute(ss2, net, l, r)) for l, r in zip(Ls, Rs)]
    b = nat.Batch([p2] * n)
    outs = b.outputs()
    unc = torch.zeros(n, dtype=torch.int32, device="cuda")
    for rep in range(2):
        b.learned_compute(net, Ls, Rs, outs, 0.5, unc)
        torch.cuda.synchronize()
        for i, (o, s) in enumerate(zip(outs, singles)):
            for k in ("depth", "disp", "flags"):
                assert np.array_equal(o[k].cpu().numpy(), s[k]), (rep, i, k)
    for x in (b, ss2, net):
        x.close()


def test_fused_inference_two_sensor_images_equals_layered_forward(nat):
    """Fused inference with batch 2 at 720x1280 against the per-layer forward."""
    import torch
    from oracle import net_oracle as no
    B, H, W = 2, 720, 1280
    rng = np.random.default_rng(77)
    x = np.zeros((B, H, W, 8), np.float32)
    x[..., :4] = rng.uniform(0, 1, (B, H, W, 4))
    bits = (no.bf16_round(x).astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    net = trained_net(nat, B * H * W)
    feats = dev(bits).view(torch.int16)
    ref = net.forward(feats).cpu().numpy()
    got = net.infer(feats)["out"].cpu().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    net.close()


def test_uneven_batch_with_sensor_slot_equals_single_pairs(orc, nat):
    """An uneven batch holding a 1280x720/D=128 slot (as in the 64-pair batch)
    equals each pair computed alone."""
    import torch
    shapes = [(320, 240, 64), (1280, 720, 128), (640, 480, 96), (848, 480, 128)]
    params, Ls, Rs = [], [], []
    for i, (W, H, D) in enumerate(shapes):
        cfg = sensor_like(W, H, D)
        params.append(cfg["params"])
        l, r = noisy_pairs(orc, cfg, [pair_seed(HELD_OUT, 300 + i)])
        Ls += l
        Rs += r
    singles = []
    for p, l, r in zip(params, Ls, Rs):
        ss = nat.SimSense(p)
        singles.append([t.cpu().numpy() for t in ss(l, r)])
        ss.close()
    b = nat.Batch(params)
    outs = b.outputs()
    for rep in range(2):
        b.compute(Ls, Rs, outs)
        torch.cuda.synchronize()
        for i, (o, s) in enumerate(zip(outs, singles)):
            for k, want in zip(("depth", "disp", "flags"), s):
                assert np.array_equal(o[k].cpu().numpy(), want), (rep, shapes[i], k)
    b.close()
