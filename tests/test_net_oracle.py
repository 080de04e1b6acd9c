"""Pins of the learned part's CPU oracle: closed forms of the convolution, the
losses and Adam, bfloat16 rounding on known values, and central finite
differences of the full loss with respect to parameters and inputs."""
import numpy as np
import pytest

from oracle import net_oracle as no


def test_param_count():
    assert no.NUM_PARAMS == 20258
    p = no.init_params(0)
    assert np.array_equal(no.flatten(no.unflatten(no.flatten(p))), no.flatten(p))


def test_conv_delta_kernel_is_a_shift():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 7, 3))
    for ky in range(3):
        for kx in range(3):
            w = np.zeros((3, 3, 3, 3))
            w[ky, kx] = np.eye(3)
            y = no.conv3x3(x, w, np.zeros(3))
            # out(y, x) = in(y + ky - 1, x + kx - 1), zero outside
            xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
            assert np.array_equal(y, xp[:, ky:ky + 5, kx:kx + 7, :])


def test_conv_constant_interior_and_bias():
    w = np.random.default_rng(1).standard_normal((3, 3, 2, 4))
    b = np.arange(4.0)
    y = no.conv3x3(np.full((1, 6, 6, 2), 2.0), w, b)
    assert np.allclose(y[0, 2, 3], 2.0 * w.sum(axis=(0, 1, 2)) + b)
    # a corner sees only the 2x2 taps that stay inside
    assert np.allclose(y[0, 0, 0], 2.0 * w[1:, 1:].sum(axis=(0, 1, 2)) + b)


def test_loss_closed_forms():
    out = np.zeros((1, 2, 2, 2))
    out[..., 0] = [[1.0, -2.0], [0.5, 3.0]]
    t = np.zeros((1, 2, 2))
    v = np.array([[[1, 0], [1, 1]]])
    total, l1, bce, g = no.loss(out, t, v)
    assert l1 == pytest.approx((1.0 + 0.5 + 3.0) / 3)
    assert bce == pytest.approx(np.log(2.0))  # every logit is 0
    assert g[0, 0, 1, 0] == 0.0 and g[0, 0, 0, 0] == pytest.approx(1 / 3)
    assert g[0, 0, 0, 1] == pytest.approx((0.5 - 1) / 4) and g[0, 0, 1, 1] == pytest.approx(0.5 / 4)


def test_adam_first_step_is_signed_lr():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -0.25, 4.0])
    m, v = np.zeros(3), np.zeros(3)
    no.adam_step(p, g, m, v, 1, 0.01)
    assert np.allclose(p, [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], atol=1e-9)


def test_adam_three_steps_hand_computed():
    """Steps 1-3 of one parameter (p0 = 0.5, lr = 0.1, gradients 1, -2, 0.5), worked
    out by hand from the update of Kingma and Ba (Algorithm 1): m_t = b1 m + (1-b1) g,
    v_t = b2 v + (1-b2) g^2, p -= lr (m_t / (1-b1^t)) / (sqrt(v_t / (1-b2^t)) + eps).
    From step 2 on the two decay rates no longer cancel, so swapping them fails."""
    p, m, v = np.array([0.5]), np.zeros(1), np.zeros(1)
    want = [  # (m, v, p) after each step
        (0.1, 0.001, 0.400000001),
        (-0.11, 0.004999, 0.43661035347207509),   # m^ = -0.11/0.19, v^ = 0.004999/0.001999
        (-0.049, 0.005244001, 0.45027941967382173),  # m^ = -0.049/0.271, v^ = 0.005244001/0.002997001
    ]
    for t, (g, (wm, wv, wp)) in enumerate(zip((1.0, -2.0, 0.5), want), 1):
        no.adam_step(p, np.array([g]), m, v, t, 0.1)
        assert m[0] == pytest.approx(wm, rel=1e-12)
        assert v[0] == pytest.approx(wv, rel=1e-12)
        assert p[0] == pytest.approx(wp, rel=1e-12)
    # the swapped decay rates give another parameter at step 2
    p2, m2, v2 = np.array([0.5]), np.zeros(1), np.zeros(1)
    for t, g in enumerate((1.0, -2.0), 1):
        no.adam_step(p2, np.array([g]), m2, v2, t, 0.1, b1=0.999, b2=0.9)
    assert abs(p2[0] - 0.43661035347207509) > 1e-3


def test_bf16_rounding_known_values():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -3.0, 1e-3, 65504.0], np.float32)
    got = no.bf16_round(vals)
    assert got[0] == 1.0 and got[1] == 1.0  # tie to even
    assert got[2] == 1 + 2 ** -6               # tie to even (upwards)
    assert got[3] == -3.0
    assert abs(got[4] - 1e-3) <= 1e-3 * 2 ** -8
    assert got[5] == 65536.0


def _total_loss(params, x, t, v):
    out, _ = no.forward(params, x)
    return no.loss(out, t, v)[0]


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    B, H, W = 1, 5, 6
    x = rng.uniform(0, 1, (B, H, W, 4))
    t = rng.uniform(-1, 1, (B, H, W))
    v = rng.random((B, H, W)) < 0.6
    params = no.init_params(7)
    params = [(w, rng.uniform(-0.1, 0.1, b.shape)) for w, b in params]
    out, acts = no.forward(params, x)
    _, _, _, g = no.loss(out, t, v)
    grads = no.backward(params, acts, g)
    flat = no.flatten(params)
    gflat = no.flatten(grads)
    h = 1e-6
    idx = rng.choice(flat.size, 40, replace=False)
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        num = (_total_loss(no.unflatten(fp), x, t, v) - _total_loss(no.unflatten(fm), x, t, v)) / (2 * h)
        assert num == pytest.approx(gflat[i], rel=1e-4, abs=1e-7), i
    # input gradient of the first layer through the chain
    w0 = params[0][0]
    dx, _, _ = no.conv3x3_backward(acts[0], w0, _layer0_dout(params, acts, g))
    for _ in range(10):
        pos = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[pos] += h
        xm[pos] -= h
        num = (_total_loss(params, xp, t, v) - _total_loss(params, xm, t, v)) / (2 * h)
        assert num == pytest.approx(dx[pos], rel=1e-4, abs=1e-7)


def _layer0_dout(params, acts, g):
    """Gradient at the output of layer 0 (before its ReLU), by running the chain down."""
    d = g
    for i in range(len(params) - 1, 0, -1):
        dx, _, _ = no.conv3x3_backward(acts[i], params[i][0], d)
        d = dx * (acts[i] > 0)
    return d


def test_features_and_combine():
    ir = np.array([[0, 255]], np.float64)
    f = no.features(ir, np.array([[10, 20]]), np.array([[-1, 40]]), np.array([[0, 64]]), 128, 234.0)
    assert np.allclose(f[0, 0], [0, 10 / 234, 1.0, 0]) and np.allclose(f[0, 1], [1, 20 / 234, 40 / 234, 0.5])
    out = np.array([[[0.5, 1.0], [0.25, -1.0], [-3.0, 2.0]]])
    assert np.allclose(no.combine(np.array([[10.0, 10.0, 2.0]]), out), [[10.5, 0.0, 0.0]])
