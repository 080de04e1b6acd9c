"""Pins of the on-device noise generator's oracle (Philox4x32-10 draws, the
gamma and normal conversions, the noise-scale knob)."""
import numpy as np
import pytest
from scipy import stats


def test_philox_known_answers(orc):
    # the known-answer vectors published with the generator (Random123)
    assert orc.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert orc.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert orc.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == \
        [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_uniform_conversion(orc):
    assert orc.u01(0) == 2.0 ** -24 and orc.u01(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    for x in (0, 511, 512, 0x80000000, 0xFFFFFFFF):
        u = orc.u01(x)
        assert 0.0 < u < 1.0 and float(np.float32(u)) == u  # exact in float32


@pytest.mark.parametrize("model,dist", [
    (1, stats.gamma(a=3.98, scale=0.254)),
    (2, stats.norm(loc=1.0, scale=0.05)),
])
def test_gain_distributions(orc, model, dist):
    g, n = orc.noise_draws(100_000, model, seed=12345, noise_stream=3)
    assert stats.kstest(g.astype(np.float64), dist.cdf).pvalue > 1e-3
    assert abs(g.mean() - dist.mean()) < 5 * dist.std() / np.sqrt(g.size)
    assert stats.kstest(n.astype(np.float64), stats.norm(loc=-0.231, scale=0.83).cdf).pvalue > 1e-3
    g0, n0 = orc.noise_draws(1000, 0, seed=12345, noise_stream=3)
    assert (g0 == 1.0).all() and np.array_equal(n0, n[:1000])


def test_counter_based_and_scale(orc):
    g, n = orc.noise_draws(5000, 1, seed=7, noise_stream=1)
    g2, n2 = orc.noise_draws(300, 1, seed=7, noise_stream=1)
    assert np.array_equal(g[:300], g2) and np.array_equal(n[:300], n2)  # depends on the pixel only
    g3, _ = orc.noise_draws(300, 1, seed=7, noise_stream=2)
    assert not np.array_equal(g2, g3)
    gz, nz = orc.noise_draws(5000, 1, seed=7, noise_stream=1, scale=0.0)
    assert (gz == 1.0).all() and (nz == 0.0).all()
    gh, nh = orc.noise_draws(5000, 1, seed=7, noise_stream=1, scale=0.5)
    assert np.allclose(gh - 1.0, 0.5 * (g.astype(np.float64) - 1.0), atol=1e-6)
    assert np.allclose(nh, 0.5 * n.astype(np.float64), atol=1e-6)
