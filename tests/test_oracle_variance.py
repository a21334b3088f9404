"""Pins of the oracle's variance estimate from the data (Sec. 3.3, Eqs. 18-21):
Poisson-noise mocks whose normalised residuals must have unit variance, the
gain and offset entering as the paper defines them, the extra weight factor
and the excluded non-positive counts."""
import numpy as np

from oracle.variance import weights_from_data


def test_poisson_mock_gives_unit_normalised_residuals():
    rng = np.random.default_rng(11)
    g, b = 2.5 * 600.0, 0.3                       # electronic gain x exposure time; subtracted sky
    rate = rng.uniform(5.0, 50.0, 200_000)        # data units: true d + b, i.e. counts / g
    k = rng.poisson(rate * g)                     # photon counts
    d = k / g - b                                 # the data as delivered (offset subtracted)
    w = weights_from_data(d, g, b)
    z2 = w * (d - (rate - b)) ** 2
    # E[(k - lam)^2 / k] = 1 + O(1/lam); the sample mean has std ~ sqrt(2 / n)
    assert abs(z2.mean() - 1.0) < 5 * np.sqrt(2.0 / len(z2)) + 2.0 / (rate.min() * g)
    # the estimate itself: s^2 = k / g^2
    assert np.allclose(1.0 / w, k / g ** 2, rtol=1e-12)


def test_gain_and_offset_maps_and_extra_factor():
    rng = np.random.default_rng(2)
    d = rng.uniform(-0.5, 3.0, (7, 9))
    g = rng.uniform(10.0, 100.0, (7, 9))
    b = rng.uniform(0.0, 1.0, (7, 9))
    extra = rng.uniform(0.0, 2.0, (7, 9))
    extra[2, 3] = 0.0                              # masked
    w = weights_from_data(d, g, b, extra)
    for i in range(7):
        for j in range(9):
            k = g[i, j] * (d[i, j] + b[i, j])
            want = extra[i, j] * g[i, j] / (d[i, j] + b[i, j]) if k > 0 else 0.0
            assert w[i, j] == want or abs(w[i, j] - want) <= 1e-15 * abs(want)
    assert w[2, 3] == 0.0
    # scalar gain/offset equal constant maps
    assert np.array_equal(weights_from_data(d, 40.0, 0.2), weights_from_data(d, np.full_like(d, 40.0),
                                                                            np.full_like(d, 0.2)))
    # doubling the gain halves the variance
    assert np.allclose(weights_from_data(d, 80.0, 0.2)[d + 0.2 > 0], 2 * weights_from_data(d, 40.0, 0.2)[d + 0.2 > 0])


def test_non_positive_counts_get_no_weight():
    d = np.array([-1.0, -0.2, 0.0, -0.2 + 1e-12, 5.0])      # counts -2.4, 0, 0.6, 3e-12, 15.6
    w = weights_from_data(d, 3.0, 0.2)
    assert np.array_equal(w[:2], [0.0, 0.0])
    assert w[2] == 3.0 / 0.2 and w[3] > 1e11 and w[4] == 3.0 / 5.2
