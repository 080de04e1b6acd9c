"""Rectification and depth registration on the GPU against the oracle, bit for bit
(both evaluate the same float32 operations in the same order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("H,W,oh,ow", [(720, 1280, 720, 1280), (61, 97, 45, 130), (1, 5, 3, 1)])
def test_rectify_matches_oracle(orc, nat, H, W, oh, ow):
    rng = np.random.default_rng(H + W)
    img = rng.integers(0, 256, (H, W)).astype(np.uint8)
    ys, xs = np.mgrid[0:oh, 0:ow].astype(np.float64)
    # a mild rotation + radial distortion, with sources leaving the image near the border
    c, s = np.cos(0.01), np.sin(0.01)
    u, v = xs - ow / 2, ys - oh / 2
    r2 = (u * u + v * v) / max(1.0, (ow / 2) ** 2)
    mx = (c * u - s * v) * (1 + 0.02 * r2) + W / 2 + rng.uniform(-0.5, 0.5, u.shape)
    my = (s * u + c * v) * (1 + 0.02 * r2) + H / 2 + rng.uniform(-0.5, 0.5, u.shape)
    mx, my = mx.astype(np.float32), my.astype(np.float32)
    got = nat.rectify(dev(img), dev(mx), dev(my)).cpu().numpy()
    assert np.array_equal(got, orc.rectify(img, mx, my))


@pytest.mark.parametrize("H,W,ow,oh", [(720, 1280, 1920, 1080), (31, 47, 50, 40)])
def test_register_matches_oracle(orc, nat, H, W, ow, oh):
    rng = np.random.default_rng(W)
    depth = rng.uniform(0.3, 4.0, (H, W)).astype(np.float32)
    depth[rng.random((H, W)) < 0.15] = 0.0
    ir = (920.0 * W / 1280, 920.0 * W / 1280, (W - 1) / 2, (H - 1) / 2)
    rgb = (1380.0 * ow / 1920, 1380.0 * ow / 1920, (ow - 1) / 2 + 3.25, (oh - 1) / 2 - 1.5)
    a = 0.02
    rt = [np.cos(a), 0.0, np.sin(a), 0.0, 1.0, 0.0, -np.sin(a), 0.0, np.cos(a), -0.015, 0.001, 0.002]
    got = nat.register_depth(dev(depth), ir, rt, rgb, ow, oh).cpu().numpy()
    ref = orc.register_depth(depth, ir, np.array(rt, np.float32), rgb, ow, oh)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert (got > 0).mean() > 0.2
