"""Pins of the oracle's image-plane source positions (Sec. 5: a position drawn
on the image plane is mapped to the source plane by the lens equation and
given to the source): the chosen image point shows the source centre's
surface brightness, the equivalence with the source-plane parametrisation,
and the dual-number gradient (which now carries d beta / d lens parameters)
against Richardson differences."""
import math

import numpy as np
import pytest

import oracle

from test_oracle_pins import T_SMALL, _fd_grad, theta_base


def probe(t, x, y, source_position):
    """Surface brightness at (x, y): a 1 x 1 image centred there, point rule."""
    s = oracle.System(1, 1, 1e-3, 1, np.ones((1, 1)), center_x=x, center_y=y, source_position=source_position)
    return oracle.render(s, t, apply_psf=False)[0, 0] / 1e-6


@pytest.mark.parametrize("xi,yi", [(0.9, 0.4), (-0.3, 1.1), (0.05, -0.7)])
def test_the_image_point_shows_the_source_centre(xi, yi):
    """With theta[10:12] an image-plane point x_I, the lens equation maps x_I onto
    the source centre, so the lensed source there is at its central brightness
    I_e e^{b_n} (surface brightness is conserved), for an SIE plus shear."""
    n = 1.3
    t = theta_base(theta_E=1.1, q_L=0.7, phi_L=0.6, gamma=0.04, phi_gamma=1.2, x_S=xi, y_S=yi, I_S=2.0, R_S=0.2,
                   n_S=n, q_S=0.6, phi_S=0.3)
    sb = probe(t, xi, yi, "image")
    assert sb == pytest.approx(2.0 * math.exp(oracle.bn(n)), rel=1e-12)
    # a nearby point is fainter (the centre is the maximum of the source)
    assert probe(t, xi + 0.01, yi, "image") < sb


def test_image_plane_equals_source_plane_at_the_mapped_centre():
    t = T_SMALL.copy()
    t[10], t[11] = 0.7, -0.45                      # an image-plane point
    ax, ay = oracle.sie_deflection(t[0], t[1], t[2], t[10], t[11])
    gx, gy = oracle.shear_deflection(t[3], t[4], t[10], t[11])
    u = t.copy()
    u[10], u[11] = t[10] - ax - gx, t[11] - ay - gy
    psf = np.exp(-0.5 * ((np.arange(5) - 2)[:, None] ** 2 + (np.arange(5) - 2)[None, :] ** 2) / 0.9)
    si = oracle.System(20, 18, 0.1, 2, psf, source_position="image")
    ss = oracle.System(20, 18, 0.1, 2, psf)
    assert np.allclose(oracle.render(si, t), oracle.render(ss, u), rtol=1e-13, atol=0)


def test_image_plane_gradient_matches_richardson_finite_differences():
    t = T_SMALL.copy()
    t[10], t[11] = 0.75, -0.4
    psf = np.exp(-0.5 * ((np.arange(5) - 2)[:, None] ** 2 + (np.arange(5) - 2)[None, :] ** 2) / 0.9)
    s0 = oracle.System(20, 18, 0.1, 2, psf, source_position="image")
    model = oracle.render(s0, t)
    rng = np.random.default_rng(9)
    d = model + 0.02 * np.max(model) * rng.standard_normal(model.shape)
    s = oracle.System(20, 18, 0.1, 2, psf, d, np.full(model.shape, 1.0 / (0.02 * np.max(model)) ** 2),
                      source_position="image")
    t[0] += 0.02; t[10] += 0.03; t[3] += 0.01
    ll, g = oracle.loglike_grad(s, t)
    assert ll == pytest.approx(oracle.loglike(s, t), rel=1e-14)
    fd = np.array([_fd_grad(s, t, k) for k in range(17)])
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd))
