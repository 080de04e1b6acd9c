"""The seeded input generator matches its stated recipe."""
import numpy as np
import pytest

from synth import CONFIGS, PairSpec, make_pair, make_shift_pair, noise_draws, pair_seed


def test_reproducible_and_seed_dependent():
    spec = PairSpec(64, 48)
    a, b, c = make_pair(spec, 1), make_pair(spec, 1), make_pair(spec, 2)
    assert np.array_equal(a.left, b.left) and np.array_equal(a.n_r, b.n_r)
    assert not np.array_equal(a.left, c.left)
    assert pair_seed(3, 7) == 3_000_007


def test_speckle_statistics():
    spec = CONFIGS["pair_1280x720_d128"]["spec"]
    p = make_pair(spec, pair_seed(1, 0))
    dots = p.left >= 150
    assert abs(dots.mean() - 0.15) < 0.005
    assert p.left[dots].max() <= 255 and p.left[~dots].min() >= 10 and p.left[~dots].max() <= 40
    assert p.left.shape == (720, 1280)


def test_field_and_warp():
    spec = PairSpec(200, 120, planes=5, dmin=4, dmax=60, noise="none")
    p = make_pair(spec, 3)
    assert p.field.min() >= 4 and p.field.max() <= 60
    # right(x) = left(x + d) by linear interpolation where x + d stays inside
    ys, xs = np.mgrid[0:120, 0:200]
    src = xs + p.field.astype(np.float64)
    inside = src <= 199
    x0 = np.floor(src).astype(int)
    f = src - x0
    x1 = np.minimum(x0 + 1, 199)
    x0 = np.minimum(x0, 199)
    interp = np.rint((1 - f) * p.left[ys, x0] + f * p.left[ys, x1])
    assert np.array_equal(p.right[inside], interp[inside].astype(np.uint8))
    # no noise in mode "none"
    assert np.all(p.gamma_l == 1) and np.all(p.n_l == 0)


def test_gauss_noise_draws():
    spec = PairSpec(300, 300, noise="gauss", sigma=4.0, gain_sd=0.05)
    g, n = noise_draws(spec, (300, 300), 5, 4)
    assert g.dtype == np.float32 and n.dtype == np.float32
    assert g.mean() == pytest.approx(1.0, abs=0.001) and g.std() == pytest.approx(0.05, rel=0.02)
    assert n.mean() == pytest.approx(0.0, abs=0.03) and n.std() == pytest.approx(4.0, rel=0.02)
    # noise scale s maps gamma -> 1 + s (gamma - 1) and n -> s n
    spec2 = PairSpec(300, 300, noise="gauss", sigma=4.0, gain_sd=0.05, noise_scale=0.5)
    g2, n2 = noise_draws(spec2, (300, 300), 5, 4)
    assert np.allclose(g2, 1 + 0.5 * (g.astype(np.float64) - 1), atol=1e-6)
    assert np.allclose(n2, 0.5 * n, atol=1e-6)


def test_shift_pair():
    left, right = make_shift_pair(50, 10, 7, seed=1)
    assert np.array_equal(right[:, :43], left[:, 7:])
