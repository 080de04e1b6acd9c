"""Pins of the rectification and registration oracle."""
import numpy as np
from scipy.ndimage import map_coordinates


def _img(H, W, seed):
    return np.random.default_rng(seed).integers(0, 256, (H, W)).astype(np.uint8)


def test_rectify_identity_shift_and_half_pixel(orc):
    img = _img(37, 53, 1)
    H, W = img.shape
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float32)
    assert np.array_equal(orc.rectify(img, xs, ys), img)
    out = orc.rectify(img, xs + 3, ys)  # integer shift; sources past the border are black
    assert np.array_equal(out[:, : W - 3], img[:, 3:]) and (out[:, W - 3:] == 0).all()
    out = orc.rectify(img, xs[:, :-1] + 0.5, ys[:, :-1])  # midpoint: the mean, ties to even
    want = np.rint((img[:, :-1].astype(np.float64) + img[:, 1:]) / 2)
    assert np.array_equal(out, want.astype(np.uint8))
    assert (orc.rectify(img, xs - 0.25 - xs, ys) == 0).all()  # x = -0.25 is outside


def test_rectify_matches_library_bilinear(orc):
    """Against scipy's order-1 map_coordinates (double precision, constant 0
    outside): equal but at float32 rounding boundaries, and never more than 1 DN."""
    img = _img(60, 80, 2)
    rng = np.random.default_rng(3)
    my = rng.uniform(-2, 61, (40, 50)).astype(np.float32)
    mx = rng.uniform(-2, 81, (40, 50)).astype(np.float32)
    out = orc.rectify(img, mx, my).astype(int)
    inside = (mx >= 0) & (my >= 0) & (mx <= 79) & (my <= 59)
    ref = map_coordinates(img.astype(np.float64), [my.astype(np.float64), mx.astype(np.float64)], order=1,
                          mode="constant", cval=0.0)
    ref = np.where(inside, np.clip(np.rint(ref), 0, 255), 0).astype(int)
    d = np.abs(out - ref)
    assert d.max() <= 1 and (d > 0).mean() < 0.01
    assert (out[~inside] == 0).all()


def test_register_identity_translation_and_zbuffer(orc):
    H, W = 30, 40
    cam = (50.0, 50.0, 19.5, 14.5)
    rng = np.random.default_rng(4)
    depth = rng.uniform(0.5, 3.0, (H, W)).astype(np.float32)
    depth[rng.random((H, W)) < 0.2] = 0.0
    ident = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)
    assert np.array_equal(orc.register_depth(depth, cam, ident, cam, W, H), depth)
    # a camera 0.1 m to the right: u' = u - f b / z (rounded), same depth
    b = 0.1
    rt = ident.copy()
    rt[9] = -b
    out = orc.register_depth(np.full((1, W), 1.0, np.float32), cam, rt, cam, W, 1)
    shift = int(round(50.0 * b / 1.0))
    assert np.array_equal(out[0, : W - shift], np.ones(W - shift, np.float32)) and (out[0, W - shift:] == 0).all()
    # two pixels landing on one: the nearer depth wins; points behind the camera vanish
    two = np.zeros((1, W), np.float32)
    two[0, 15], two[0, 20], two[0, 30] = 1.0, 0.5, 2.0  # 15 - 5 = 10, 20 - 10 = 10, 30 - 2.5 -> 28 (ties to even)
    out = orc.register_depth(two, cam, rt, cam, W, 1)
    assert out[0, 10] == 0.5 and out[0, 28] == 2.0 and np.count_nonzero(out) == 2
    behind = ident.copy()
    behind[11] = -10.0
    assert (orc.register_depth(depth, cam, behind, cam, W, H) == 0).all()
