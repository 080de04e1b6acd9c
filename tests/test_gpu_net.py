"""GPU checks of the learned surrogate against the fp64 CPU oracle.

The GPU stores weights, activations and gradients in bf16 and accumulates in
fp32.  Each stage is checked element by element against the oracle fed the
GPU's own bf16 inputs of that stage (read back from the net), with a bound
derived per element from the arithmetic: fp32 accumulation error of the sum
(2 K u32 times the sum of the absolute terms) plus one bf16 rounding (2^-8
relative) where the GPU stores bf16.
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


U32 = 2.0 ** -24  # fp32 unit roundoff
UBF = 2.0 ** -8   # bf16 unit roundoff (8 significant bits)


def bf(bits):
    """bf16 bit patterns (uint16) as float64 values."""
    return (np.ascontiguousarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def gpu_layer_inputs(nat, net, xbits, B, H, W):
    """The four layers' inputs as the GPU holds them (bf16 values) and its fp32 output."""
    P = B * H * W
    xs = [bf(xbits)[..., :4]]
    for l in range(3):
        xs.append(bf(net.read_tensor(nat.NET_ACTIVATION, l, P)).reshape(B, H, W, 32))
    out = net.read_tensor(nat.NET_OUTPUT, 3, P).reshape(B, H, W, 2).astype(np.float64)
    return xs, out


def check_forward_layers(xs, out, wq, bq):
    """Each layer against the oracle fed that layer's own GPU input, element by
    element.  A layer sums K = 9 Cin products and the bias in fp32; whatever the
    order, that sum is within 2 K u32 sum|terms| of the exact one (the factor 2
    covers a matrix core that does not round to nearest at every step), and a
    stored activation is that sum, ReLU'd, rounded once more to bf16."""
    for l in range(4):
        z = no.conv3x3(xs[l], wq[l], bq[l])
        mag = no.conv3x3(np.abs(xs[l]), np.abs(wq[l]), np.abs(bq[l]))
        e = 2 * (9 * xs[l].shape[-1] + 1) * U32 * mag
        if l < 3:
            got, ref = xs[l + 1], np.maximum(z, 0.0)
            bad = np.abs(got - ref) > 1.01 * UBF * np.abs(got) + e
        else:
            got, ref = out, z
            bad = np.abs(got - ref) > e
        assert not bad.any(), (l, int(bad.sum()), np.abs(got - ref)[bad][:4], e[bad][:4])


def quantised(params):
    """The weights as the GPU uses them (bf16) and its fp32 biases, as float64."""
    return ([no.bf16_round(w) for w, _ in params], [b.astype(np.float32).astype(np.float64) for _, b in params])


@pytest.mark.parametrize("B,H,W", [(1, 16, 16), (2, 13, 37), (1, 1, 5), (3, 9, 64)])
def test_forward_layer_by_layer_matches_oracle(nat, B, H, W):
    import torch
    x, params, _, _ = random_case(B * 1000 + H * 10 + W, B, H, W)
    net = nat.Net(B * H * W, seed=1)
    net.set_state(no.flatten(params))
    xbits = bf16_bits(x)
    net.forward(dev(xbits).view(torch.int16))
    torch.cuda.synchronize()
    xs, out = gpu_layer_inputs(nat, net, xbits, B, H, W)
    check_forward_layers(xs, out, *quantised(params))
    net.close()


@pytest.mark.parametrize("B,H,W", [(2, 12, 40), (1, 37, 150)])
def test_training_step_layer_by_layer_matches_oracle(nat, B, H, W):
    """One training step, every tensor element by element against the oracle fed
    the GPU's own inputs of that stage: forward layers, the loss gradient at the
    output, the backward-data gradients (with their ReLU masks), and the weight
    and bias gradients (sums over the batch's pixels in fp32: within
    2 P u32 sum|terms| of the exact sum).  The second size leaves partial
    convolution windows (64 columns x 16 rows) and backward-weight strips (32
    columns) on both image edges."""
    import torch
    P = B * H * W
    x, params, t, v = random_case(11 + H, B, H, W)
    net = nat.Net(P, seed=3)
    flat0 = no.flatten(params).astype(np.float32)
    net.set_state(flat0)
    xbits = bf16_bits(x)
    net.train_step(dev(xbits).view(torch.int16), dev(t.astype(np.float32)), dev(v.astype(np.uint8)), 1e-3)
    torch.cuda.synchronize()
    g_gpu = net.get_grads().astype(np.float64)
    wq, bq = quantised(no.unflatten(flat0.astype(np.float64)))
    xs, out = gpu_layer_inputs(nat, net, xbits, B, H, W)
    check_forward_layers(xs, out, wq, bq)
    # loss gradient at the output, from the GPU's own fp32 output: the residual
    # channel is sign(r - t) v / n_valid, the logit channel (sigmoid(z) - v) / P,
    # each evaluated in fp32 (a few u32 of the sigmoid, absolute 8 u32 / P at most)
    # and rounded to bf16
    dy3 = bf(net.read_tensor(nat.NET_OUTPUT_GRAD, 3, P)).reshape(B, H, W, 16)
    assert np.all(dy3[..., 2:] == 0)
    _, _, _, gref = no.loss(out, t.astype(np.float32).astype(np.float64), v)
    bad = np.abs(dy3[..., :2] - gref) > 1.01 * UBF * np.maximum(np.abs(dy3[..., :2]), np.abs(gref)) + 8 * U32 / P
    assert not bad.any(), int(bad.sum())
    dys = {3: dy3[..., :2]}
    for l in range(3):
        dys[l] = bf(net.read_tensor(nat.NET_OUTPUT_GRAD, l, P)).reshape(B, H, W, 32)
    # backward-data: the gradient at layer l-1's output from layer l's output gradient,
    # K = 9 Cout_l products per element, then the ReLU mask and the bf16 rounding
    for l in (3, 2, 1):
        dx, _, _ = no.conv3x3_backward(xs[l], wq[l], dys[l])
        ref = dx * (xs[l] > 0)
        mag = no.conv3x3_backward(np.abs(xs[l]), np.abs(wq[l]), np.abs(dys[l]))[0]
        e = 2 * 9 * dys[l].shape[-1] * U32 * mag
        got = dys[l - 1]
        assert np.all(got[xs[l] <= 0] == 0), l
        bad = np.abs(got - ref) > 1.01 * UBF * np.abs(got) + e
        assert not bad.any(), (l, int(bad.sum()))
    # weight and bias gradients
    o = 0
    for l, (ci, co) in enumerate(no.LAYERS):
        _, dw, db = no.conv3x3_backward(xs[l], wq[l], dys[l])
        _, mw, mb = no.conv3x3_backward(np.abs(xs[l]), np.abs(wq[l]), np.abs(dys[l]))
        nw = 9 * ci * co
        gw = g_gpu[o:o + nw].reshape(3, 3, ci, co)
        gb = g_gpu[o + nw:o + nw + co]
        o += nw + co
        bad_w = np.abs(gw - dw) > 2 * P * U32 * mw
        bad_b = np.abs(gb - db) > 2 * P * U32 * mb
        assert not bad_w.any(), (l, int(bad_w.sum()), np.abs(gw - dw).max())
        assert not bad_b.any(), (l, int(bad_b.sum()))
    net.close()


def test_adam_steps_match_oracle(nat):
    """Three training steps: after each, the GPU's parameters and moments equal the
    oracle's Adam update (fp64) applied to the GPU's state before the step and the
    GPU's gradient of the step, element by element.  The GPU holds the
    hyperparameters as float32 values (1 - float32(0.999) is 1.3e-5 away from
    0.001), so the oracle is given those values.  Bounds from the fp32 operations:
    a moment is two products and a sum (within 4 u32 of the sum of its absolute
    terms, which can be far above the moment itself when the two terms cancel);
    the update step m^ / (sqrt(v^) + eps) carries the moments' relative errors
    (all of m's, half of v's) plus a few correctly rounded operations (10 u32), and
    the parameter is one more subtraction (2 u32 of the operands)."""
    import torch
    B, H, W = 1, 10, 24
    x, params, t, v = random_case(31, B, H, W)
    net = nat.Net(B * H * W, seed=3)
    net.set_state(no.flatten(params).astype(np.float32))
    rng = np.random.default_rng(4)
    lr = 2e-3
    p_prev, m_prev, v_prev, step = net.get_state()
    assert step == 0
    for k in range(1, 4):
        xk = x.copy()
        xk[..., :4] = rng.uniform(0, 1, (B, H, W, 4))
        net.train_step(dev(bf16_bits(xk)).view(torch.int16), dev(t.astype(np.float32)), dev(v.astype(np.uint8)), lr)
        torch.cuda.synchronize()
        g = net.get_grads().astype(np.float64)
        p1, m1, v1, step = net.get_state()
        assert step == k
        pr, mr, vr = (a.astype(np.float64).copy() for a in (p_prev, m_prev, v_prev))
        f32 = lambda x: float(np.float32(x))
        b1, b2 = f32(0.9), f32(0.999)
        no.adam_step(pr, g, mr, vr, k, f32(lr), b1=b1, b2=b2, eps=f32(1e-8))
        m0, v0, p0 = (a.astype(np.float64) for a in (m_prev, v_prev, p_prev))
        tol_m = 4 * U32 * (np.abs(b1 * m0) + np.abs((1 - b1) * g))
        tol_v = 4 * U32 * (np.abs(b2 * v0) + np.abs((1 - b2) * g * g))
        rel_step = tol_m / np.maximum(np.abs(mr), 1e-300) + 0.5 * tol_v / np.maximum(np.abs(vr), 1e-300) + 10 * U32
        tol_p = 2 * U32 * np.abs(p0) + rel_step * np.abs(p0 - pr) + 1e-30
        assert np.all(np.abs(m1 - mr) <= tol_m), (k, np.abs(m1 - mr).max())
        assert np.all(np.abs(v1 - vr) <= tol_v), (k, np.abs(v1 - vr).max())
        bad = np.abs(p1 - pr) > tol_p
        if bad.any():
            i = int(np.argmax(np.abs(p1 - pr) / tol_p))
            raise AssertionError(f"step {k}: {int(bad.sum())} parameters off; worst {i}: gpu {p1[i]!r} oracle "
                                 f"{pr[i]!r} p0 {p0[i]!r} m {m1[i]!r} v {v1[i]!r} g {g[i]!r} "
                                 f"err/update {abs(p1[i] - pr[i]) / max(abs(p0[i] - pr[i]), 1e-300):.3e}")
        p_prev, m_prev, v_prev = p1, m1, v1
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


@pytest.mark.parametrize("paths,census_mode,p2,D", [(2, 0, 86, 64), (4, 1, 150, 96), (8, 0, 200, 128)])
def test_features_and_learned_path_match_oracle(nat, orc, paths, census_mode, p2, D):
    """The learned depth path link by link: the features pass equals the oracle's
    features bit for bit (float32 quotients rounded to bf16, as the kernel does),
    the net on them matches the oracle layer by layer within the per-element
    bounds, and the path's final disparity (whose fused kernel builds the features
    itself from the selection outputs) equals the oracle's combination (float32)
    and median of the sub-pixel map and the net output, bit for bit.  Besides the
    2-path form, other path counts, the full census and other penalties change the
    feature scale Smax = paths x (bits + P2) (234, 848, 1848 here) and the
    disparity range that the in-kernel feature quotients cover."""
    import torch
    from synth import PairSpec, make_pair
    W, H = 160, 96
    params2 = dict(width=W, height=H, max_disp=D, census_w=7, census_h=9, census_mode=census_mode, p1=7, p2=p2,
                   uniqueness_pct=10, lr_max_diff=1, num_paths=paths, median=3, subpixel=1, focal_px=400.0,
                   baseline_m=0.055)
    pr = make_pair(PairSpec(W, H, planes=4, dmin=4, dmax=min(50, D - 4), noise="gauss", sigma=3.0), 17)
    L = orc.ir_noise(pr.left, pr.gamma_l, pr.n_l)
    R = orc.ir_noise(pr.right, pr.gamma_r, pr.n_r)
    ref2 = orc.sgm(params2, L, R)
    smax = paths * ((62 if census_mode else 31) + p2)
    feats_ref = no.features(L, ref2.s1, ref2.s2, ref2.dint, D, float(smax), dtype=np.float32)
    ss = nat.SimSense(params2)
    g = ss.compute_all(dev(L), dev(R), features=True)
    fg = g["features"].cpu().numpy().view(np.uint16)
    assert np.all(fg[..., 4:] == 0)
    assert np.array_equal(fg[..., :4], bf16_bits(feats_ref))
    d2 = g["disp_sub"].cpu().numpy()
    assert np.max(np.abs(d2.astype(np.float64) - ref2.dsub)) <= 1e-5

    rng = np.random.default_rng(2)
    params = [(w, rng.uniform(-0.05, 0.05, b.shape)) for w, b in no.init_params(4)]
    net = nat.Net(W * H, seed=0)
    net.set_state(no.flatten(params))
    fbits = np.ascontiguousarray(fg.reshape(1, H, W, 8))
    net.forward(dev(fbits).view(torch.int16))
    torch.cuda.synchronize()
    xs, out = gpu_layer_inputs(nat, net, fbits, 1, H, W)
    check_forward_layers(xs, out, *quantised(params))
    res = nat.learned_compute(ss, net, dev(L), dev(R), extras=True)
    torch.cuda.synchronize()
    assert np.array_equal(res["disp_sub"].cpu().numpy(), d2)
    want = orc.median3(no.combine(d2, out[0].astype(np.float32), dtype=np.float32)).astype(np.float32)
    assert np.array_equal(res["disp"].cpu().numpy(), want)
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
