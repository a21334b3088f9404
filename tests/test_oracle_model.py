"""Pins of the oracle's general models (Sec. 5: several lenses and light
components, a flat sky, free centres): the base model is the 17-parameter one,
the deflections of several lenses add, an off-centre lens is the centred one
translated, a flat sky is a constant, and log L follows Eq. 17."""
import numpy as np
import pytest

import oracle

from test_oracle_pins import T_SMALL


def system(H=20, W=18, d=0.1, cx=0.0, cy=0.0, data=None, weight=None):
    psf = np.exp(-0.5 * ((np.arange(5) - 2)[:, None] ** 2 + (np.arange(5) - 2)[None, :] ** 2) / 0.9)
    return oracle.System(H, W, d, 2, psf, data, weight, center_x=cx, center_y=cy)


def base_params(t):
    """The 17-parameter point as a general model: SIE at the origin, shear, host
    light at the origin (image plane), source (source plane)."""
    return np.concatenate([[0.0, 0.0], t[0:3], t[3:5], [0.0, 0.0], t[5:10], t[10:17]])


BASE = oracle.Model(1, ["image", "source"], shear=True)


def test_the_base_model_is_the_17_parameter_model():
    s = system()
    assert BASE.n_params == 21
    # the deflections are summed before they are subtracted: equal to rounding
    assert np.allclose(oracle.render_model(s, BASE, base_params(T_SMALL)), oracle.render(s, T_SMALL), rtol=1e-14,
                       atol=0)


def test_deflections_of_several_lenses_add():
    """SIE deflection is linear in theta_E: two coincident SIEs of theta_E/2 are
    one of theta_E."""
    s = system()
    two = oracle.Model(2, ["image", "source"], shear=True)
    p = base_params(T_SMALL)
    half = p[0:5].copy()
    half[2] *= 0.5
    q = np.concatenate([half, half, p[5:]])
    assert np.allclose(oracle.render_model(s, two, q), oracle.render_model(s, BASE, p), rtol=1e-12, atol=0)


def test_an_off_centre_lens_is_the_centred_one_translated():
    """Without shear (which acts about the origin), moving the lens, the host
    light, the source and the grid by the same offset leaves the image alone."""
    m = oracle.Model(1, ["image", "source"], shear=False)
    p = np.concatenate([[0.0, 0.0], T_SMALL[0:3], [0.0, 0.0], T_SMALL[5:10], T_SMALL[10:17]])
    off = np.array([0.37, -0.21])
    q = p.copy()
    q[0:2] += off
    q[5:7] += off
    q[12:14] += off
    a = oracle.render_model(system(), m, p)
    b = oracle.render_model(system(cx=off[0], cy=off[1]), m, q)
    assert np.allclose(a, b, rtol=1e-9, atol=1e-12 * np.max(a))


def test_flat_sky_and_log_likelihood():
    sky_model = oracle.Model(0, ["image"], shear=False, sky=True)
    p = np.array([0.0, 0.0, 0.0, 0.3, 1.0, 0.8, 0.2, 2.5])    # a dark Sersic and the sky
    img = oracle.render_model(system(), sky_model, p)
    assert np.allclose(img, 2.5 * 0.1 ** 2, rtol=1e-14, atol=0)
    rng = np.random.default_rng(6)
    d, w = rng.random(360), rng.uniform(0.5, 2.0, 360)
    assert oracle.loglike_model(system(data=d, weight=w), sky_model, p) == pytest.approx(
        -0.5 * np.sum(w * (d - 0.025) ** 2), rel=1e-13)
    # the base model's log L is the plain one
    s = system(data=d, weight=w)
    assert oracle.loglike_model(s, BASE, base_params(T_SMALL)) == pytest.approx(oracle.loglike(s, T_SMALL),
                                                                             rel=1e-14)
