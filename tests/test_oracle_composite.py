"""Pins of the oracle's composite models (Sec. 5: a base model plus extra Sersic
components and a flat sky): one component without sky is the plain model, the
image is linear in the components, a flat sky survives the PSF as a constant,
and log L follows Eq. 17 on the summed image."""
import numpy as np
import pytest

import oracle

from test_oracle_pins import T_SMALL


def system(data=None, weight=None):
    psf = np.exp(-0.5 * ((np.arange(5) - 2)[:, None] ** 2 + (np.arange(5) - 2)[None, :] ** 2) / 0.9)
    return oracle.System(20, 18, 0.1, 2, psf, data, weight)


def test_one_component_without_sky_is_the_plain_model():
    rng = np.random.default_rng(1)
    s = system(rng.random(360), rng.uniform(0.5, 2.0, 360))
    assert np.array_equal(oracle.render_composite(s, T_SMALL[None]), oracle.render(s, T_SMALL))
    assert oracle.loglike_composite(s, T_SMALL[None]) == pytest.approx(oracle.loglike(s, T_SMALL), rel=1e-15)


def test_components_add_and_amplitudes_are_linear():
    s = system()
    half = T_SMALL.copy()
    half[5] *= 0.5
    half[12] *= 0.5
    two = oracle.render_composite(s, np.stack([half, half]))
    assert np.allclose(two, oracle.render(s, T_SMALL), rtol=1e-13, atol=0)
    other = T_SMALL.copy()
    other[12:17] = [0.4, 0.1, 2.5, 0.5, 0.2]
    other[5] = 0.0
    both = oracle.render_composite(s, np.stack([T_SMALL, other]))
    assert np.allclose(both, oracle.render(s, T_SMALL) + oracle.render(s, other), rtol=1e-13, atol=1e-18)


def test_flat_sky_stays_flat_through_the_psf():
    s = system()
    dark = T_SMALL.copy()
    dark[5] = dark[12] = 0.0
    img = oracle.render_composite(s, dark[None], sky=3.0)
    assert np.allclose(img, 3.0 * 0.1 ** 2, rtol=1e-14, atol=0)
    d = np.random.default_rng(2).random(360)
    w = np.random.default_rng(3).uniform(0.5, 2.0, 360)
    sw = system(d, w)
    assert oracle.loglike_composite(sw, dark[None], sky=3.0) == pytest.approx(
        -0.5 * np.sum(w * (d - 0.03) ** 2), rel=1e-13)


def test_bands_add_their_log_likelihoods():
    rng = np.random.default_rng(4)
    s1 = system(rng.random(360), rng.uniform(0.5, 2.0, 360))
    s0 = system(rng.random(360), np.zeros(360))                  # a band without weights adds nothing
    t = T_SMALL[None]
    one = oracle.loglike_composite(s1, t, 0.2)
    assert oracle.loglike_multiband([s1, s1], [t, t], [0.2, 0.2]) == pytest.approx(2 * one, rel=1e-15)
    assert oracle.loglike_multiband([s1, s0], [t, t], [0.2, 0.2]) == pytest.approx(one, rel=1e-15)
