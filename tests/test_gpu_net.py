"""GPU checks of the learned surrogate against the fp64 CPU oracle.

The GPU stores weights, activations and gradients in bf16 and accumulates in
fp32; the oracle repeats the same bf16 roundings of weights and activations and
computes in fp64.  Rounding-boundary flips and fp32 accumulation order leave
relative differences of the order of the bf16 epsilon (2^-8), which is the
tolerance used here.
"""
import numpy as np
import pytest

from oracle import net_oracle as no

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nat():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_11924_amd.native as n
    return n


def bf16_bits(a):
    f = no.bf16_round(a).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def random_case(seed, B, H, W):
    rng = np.random.default_rng(seed)
    x = np.zeros((B, H, W, 8))
    x[..., :4] = rng.uniform(0, 1, (B, H, W, 4))
    params = no.init_params(seed)
    params = [(w, rng.uniform(-0.05, 0.05, b.shape)) for w, b in params]
    t = rng.uniform(-1.5, 1.5, (B, H, W))
    v = rng.random((B, H, W)) < 0.7
    return x, params, t, v


def test_forward_matches_oracle(nat):
    import torch
    for seed, (B, H, W) in enumerate([(1, 16, 16), (2, 13, 37), (1, 1, 5), (3, 9, 64)]):
        x, params, _, _ = random_case(seed, B, H, W)
        net = nat.Net(B * H * W, seed=1)
        net.set_state(no.flatten(params))
        out = net.forward(dev(bf16_bits(x)).view(torch.int16)).cpu().numpy().astype(np.float64)
        # the oracle with the GPU's roundings; the GPU keeps fp32 params and rounds weights to bf16
        qparams = [(no.bf16_round(w), b.astype(np.float32).astype(np.float64)) for w, b in params]
        ref, _ = no.forward(qparams, no.bf16_round(x)[..., :4], round_bf16=True)
        err = np.abs(out - ref)
        scale = np.abs(ref).mean() + 1e-3
        assert err.max() <= 4e-2 * scale + 2e-2 * np.abs(ref).max(), (seed, err.max(), scale)
        assert err.mean() <= 1e-2 * scale, (seed, err.mean(), scale)
        net.close()


def test_gradients_and_adam_match_oracle(nat):
    import torch
    B, H, W = 2, 12, 40
    x, params, t, v = random_case(11, B, H, W)
    net = nat.Net(B * H * W, seed=3)
    flat0 = no.flatten(params).astype(np.float32)
    net.set_state(flat0)
    lr = 1e-3
    loss = net.train_step(dev(bf16_bits(x)).view(torch.int16), dev(t.astype(np.float32)), dev(v.astype(np.uint8)), lr)
    torch.cuda.synchronize()
    g_gpu = net.get_grads().astype(np.float64)
    p1, m1, v1, step = net.get_state()
    assert step == 1
    qparams = [(no.bf16_round(w), b.astype(np.float32).astype(np.float64)) for w, b in no.unflatten(flat0.astype(np.float64))]
    out, acts = no.forward(qparams, no.bf16_round(x)[..., :4], round_bf16=True)
    total, l1, bce, gout = no.loss(out, t, v)
    grads = no.flatten(no.backward(qparams, acts, gout))
    # per layer: relative error of the gradient vector
    o = 0
    for ci, co in no.LAYERS:
        for n in (9 * ci * co, co):
            a, b = g_gpu[o:o + n], grads[o:o + n]
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
            cos = float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))
            assert rel <= 3e-2 and cos >= 0.999, (ci, co, n, rel, cos)
            o += n
    # loss of the forward pass (computed in fp32 from the GPU output)
    lv = loss.cpu().numpy()
    assert lv[1] == pytest.approx(l1, rel=2e-2) and lv[2] == pytest.approx(bce, rel=2e-2)
    # Adam applied to the GPU's own gradient
    p_ref = flat0.astype(np.float64).copy()
    m_ref, v_ref = np.zeros_like(p_ref), np.zeros_like(p_ref)
    no.adam_step(p_ref, g_gpu, m_ref, v_ref, 1, lr)
    assert np.allclose(p1, p_ref, rtol=1e-5, atol=1e-7)
    assert np.allclose(m1, m_ref, rtol=1e-5, atol=1e-12)
    net.close()


def test_training_lowers_loss_and_resume_is_exact(nat):
    import torch
    B, H, W = 4, 32, 48
    rng = np.random.default_rng(5)
    x = np.zeros((B, H, W, 8))
    x[..., :4] = rng.uniform(0, 1, (B, H, W, 4))
    # a learnable target: residual and validity are simple functions of the features
    t = (x[..., 1] - x[..., 2]) * 2.0
    v = x[..., 3] > 0.3
    xb = dev(bf16_bits(x)).view(torch.int16)
    tt, vv = dev(t.astype(np.float32)), dev(v.astype(np.uint8))
    net = nat.Net(B * H * W, seed=7)
    losses = [float(net.train_step(xb, tt, vv, 3e-3).cpu()[0]) for _ in range(60)]
    assert losses[-1] < 0.6 * losses[0], losses[::10]
    # checkpoint, continue, restore, continue again: bitwise identical
    state = net.get_state()
    a = [net.train_step(xb, tt, vv, 3e-3).cpu().numpy() for _ in range(3)]
    pa = net.get_state()[0]
    net.set_state(state[0], state[1], state[2], state[3])
    b = [net.train_step(xb, tt, vv, 3e-3).cpu().numpy() for _ in range(3)]
    pb = net.get_state()[0]
    assert all(np.array_equal(u, w) for u, w in zip(a, b))
    assert np.array_equal(pa, pb)
    net.close()


def test_features_and_learned_path_match_oracle(nat, orc):
    import torch
    from synth import PairSpec, make_pair
    W, H, D = 160, 96, 64
    params2 = dict(width=W, height=H, max_disp=D, census_w=7, census_h=9, census_mode=0, p1=7, p2=86,
                   uniqueness_pct=10, lr_max_diff=1, num_paths=2, median=3, subpixel=1, focal_px=400.0,
                   baseline_m=0.055)
    pr = make_pair(PairSpec(W, H, planes=4, dmin=4, dmax=50, noise="gauss", sigma=3.0), 17)
    L = orc.ir_noise(pr.left, pr.gamma_l, pr.n_l)
    R = orc.ir_noise(pr.right, pr.gamma_r, pr.n_r)
    ref2 = orc.sgm(params2, L, R)
    smax = 2 * (31 + 86)
    feats_ref = no.features(L.astype(np.float64), ref2.s1, ref2.s2, ref2.dint, D, float(smax))
    ss = nat.SimSense(params2)
    g = ss.compute_all(dev(L), dev(R), features=True)
    fg = g["features"].cpu().numpy().view(np.uint16)
    fgf = (fg.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    assert np.all(fgf[..., 4:] == 0)
    assert np.allclose(fgf[..., :4], no.bf16_round(feats_ref), rtol=2 ** -8, atol=0)

    rng = np.random.default_rng(2)
    params = [(w, rng.uniform(-0.05, 0.05, b.shape)) for w, b in no.init_params(4)]
    net = nat.Net(W * H, seed=0)
    net.set_state(no.flatten(params))
    out = nat.learned_compute(ss, net, dev(L), dev(R), extras=True)
    torch.cuda.synchronize()
    qparams = [(no.bf16_round(w), b.astype(np.float32).astype(np.float64)) for w, b in params]
    o_ref, _ = no.forward(qparams, no.bf16_round(feats_ref)[None], round_bf16=True)
    disp_ref = orc.median3(no.combine(ref2.dsub, o_ref[0]))
    dg = out["disp"].cpu().numpy().astype(np.float64)
    agree = (dg > 0) == (disp_ref > 0)
    assert agree.mean() >= 0.99
    both = (dg > 0) & (disp_ref > 0)
    assert np.mean(np.abs(dg[both] - disp_ref[both]) <= 0.05) >= 0.99
    ss.close()
    net.close()


def test_learned_path_features_built_in_the_net_equal_the_features_pass(nat, orc):
    """The learned path's net builds its input features from the selection
    outputs; the result must equal the net run on the features pass's output
    (then the median), bit for bit, for one pair and for a batch."""
    import torch
    from synth import PairSpec, make_pair
    W, H, D = 150, 70, 64
    params2 = dict(width=W, height=H, max_disp=D, census_w=7, census_h=9, census_mode=0, p1=7, p2=86,
                   uniqueness_pct=10, lr_max_diff=1, num_paths=2, median=3, subpixel=1, focal_px=400.0,
                   baseline_m=0.055)
    rng = np.random.default_rng(5)
    params = [(w, rng.uniform(-0.05, 0.05, b.shape)) for w, b in no.init_params(4)]
    net = nat.Net(3 * W * H, seed=0)
    net.set_state(no.flatten(params))
    ss = nat.SimSense(params2)
    Ls, Rs, refs = [], [], []
    for seed in (21, 22, 23):
        pr = make_pair(PairSpec(W, H, planes=4, dmin=4, dmax=50, noise="gauss", sigma=3.0), seed)
        L, R = dev(orc.ir_noise(pr.left, pr.gamma_l, pr.n_l)), dev(orc.ir_noise(pr.right, pr.gamma_r, pr.n_r))
        out = nat.learned_compute(ss, net, L, R, extras=True)
        f = out["features"].view(torch.int16).reshape(1, H, W, 8).contiguous()
        m = net.infer(f, d2_sub=out["disp_sub"].reshape(1, H, W), raw=False)["masked"]
        torch.cuda.synchronize()
        ref = orc.median3(m[0].cpu().numpy().astype(np.float64)).astype(np.float32)
        assert np.array_equal(out["disp"].cpu().numpy(), ref), seed
        Ls.append(L)
        Rs.append(R)
        refs.append(out["disp"].cpu().numpy())
    b = nat.Batch([params2] * 3)
    outs = b.outputs()
    unc = torch.zeros(3, dtype=torch.int32, device="cuda")
    b.learned_compute(net, Ls, Rs, outs, 0.5, unc)
    torch.cuda.synchronize()
    for o, r in zip(outs, refs):
        assert np.array_equal(o["disp"].cpu().numpy(), r)
    b.close()
    ss.close()
    net.close()


@pytest.mark.parametrize("B,H,W", [(2, 200, 250), (1, 5, 7), (3, 91, 81), (1, 1, 300), (1, 181, 1)])
def test_fused_inference_equals_layered_forward(nat, B, H, W):
    """The fused kernel (row-strip LDS rings, several strips and row segments
    with ragged tails) gives the per-layer forward's outputs bit for bit, and
    its combination and uncertainty counts equal a host recomputation."""
    import torch
    x, params, _, _ = random_case(100 + B * H + W, B, H, W)
    net = nat.Net(B * H * W, seed=3)
    net.set_state(no.flatten(params))
    feats = dev(bf16_bits(x)).view(torch.int16)
    ref = net.forward(feats).cpu().numpy()
    rng = np.random.default_rng(H * W)
    d2 = rng.uniform(-2.0, 40.0, (B, H, W)).astype(np.float32)
    unc = torch.full((B,), 5, dtype=torch.int32, device="cuda")
    tau = 0.3
    got = net.infer(feats, d2_sub=dev(d2), tau=tau, uncertain=unc)
    out = got["out"].cpu().numpy()
    assert np.array_equal(out.view(np.uint32), ref.view(np.uint32))
    d = (d2 + ref[..., 0]).astype(np.float32)
    ok = (ref[..., 1] > 0) & (d > 0)
    assert np.array_equal(got["masked"].cpu().numpy(), np.where(ok, d, np.float32(0)))
    assert np.array_equal(got["flags"].cpu().numpy(), np.where(ok, 7, 0).astype(np.uint8))
    want = 5 + (np.abs(ref[..., 1]) < tau).reshape(B, -1).sum(1)
    assert np.array_equal(unc.cpu().numpy(), want)
    # outputs are optional: raw only, then the combination only
    assert "masked" not in net.infer(feats)
    only = net.infer(feats, d2_sub=dev(d2), raw=False)
    assert "out" not in only and torch.equal(only["masked"], got["masked"])
    net.close()
