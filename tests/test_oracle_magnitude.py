"""Pins of the oracle's magnitude parametrisation of the Sersic amplitudes
(Sec. 4.1: I_0 is chosen so that a component has a given total magnitude):
the closed-form total flux against numerical integration of the profile, the
total flux of a rendered image, the equivalence with the intensity
parametrisation, and the dual-number gradient (which now carries d I_e / d n
and d I_e / d R_e) against Richardson differences."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle

from test_oracle_pins import T_SMALL, _fd_grad, theta_base


@pytest.mark.parametrize("m,Re,n,zp", [(22.3, 0.2, 1.7, 25.0), (23.0, 0.35, 4.0, 26.5), (18.0, 0.05, 0.5, 20.0),
                                       (25.5, 1.5, 8.0, 25.5), (21.0, 0.3, 0.25, 24.0)])
def test_flux_of_the_profile_is_the_magnitude(m, Re, n, zp):
    Ie = oracle.intensity_from_magnitude(m, Re, n, zp)
    b = oracle.bn(n)
    # radial integral of I(R) 2 pi R with R/R_e = t^n: no kink at the centre
    f = lambda t: Ie * math.exp(-b * (t - 1.0)) * 2.0 * math.pi * (Re * t ** n) * Re * n * t ** (n - 1.0)
    F = integrate.quad(f, 0.0, math.inf, limit=400, epsabs=0.0, epsrel=1e-13)[0]
    assert F == pytest.approx(10.0 ** (-0.4 * (m - zp)), rel=1e-10)
    # half of it inside R_e (b_n is the half-light constant)
    half = integrate.quad(f, 0.0, 1.0, limit=400, epsabs=0.0, epsrel=1e-13)[0]
    assert half == pytest.approx(0.5 * F, rel=1e-10)


def test_rendered_image_carries_the_total_flux():
    """An unlensed elliptical n = 1 source well inside a 200 x 200 grid: the sum
    of the pixel luminosities is its total flux 10^(-0.4 (m - zp))."""
    m, zp = 21.7, 24.0
    t = theta_base(I_H=60.0, R_H=0.5, x_S=0.05, y_S=-0.03, I_S=m, R_S=0.2, n_S=1.0, q_S=0.7, phi_S=0.4)
    s = oracle.System(200, 200, 0.05, 4, np.ones((1, 1)), amplitude="magnitude", zero_point=zp)
    img = oracle.render(s, t, apply_psf=False)
    assert img.sum() == pytest.approx(10.0 ** (-0.4 * (m - zp)), rel=2e-5)


def test_magnitudes_equal_the_converted_intensities():
    zp = 25.0
    t = T_SMALL.copy()
    t[5], t[12] = 19.5, 22.0                          # magnitudes
    u = t.copy()
    u[5] = oracle.intensity_from_magnitude(t[5], t[6], t[7], zp)
    u[12] = oracle.intensity_from_magnitude(t[12], t[13], t[14], zp)
    sm = oracle.System(20, 18, 0.1, 2, np.ones((3, 3)), amplitude="magnitude", zero_point=zp)
    si = oracle.System(20, 18, 0.1, 2, np.ones((3, 3)))
    assert np.allclose(oracle.render(sm, t), oracle.render(si, u), rtol=1e-13, atol=0)
    # one magnitude brighter is 10^0.4 times the flux
    t2 = t.copy(); t2[12] -= 1.0
    assert oracle.intensity_from_magnitude(t2[12], t[13], t[14], zp) == pytest.approx(10 ** 0.4 * u[12], rel=1e-14)


def test_magnitude_gradient_matches_richardson_finite_differences():
    zp = 25.0
    t = T_SMALL.copy()
    t[5], t[12] = 21.0, 22.5
    s0 = oracle.System(20, 18, 0.1, 2, np.exp(-0.5 * ((np.arange(5) - 2)[:, None] ** 2 + (np.arange(5) - 2)[None, :] ** 2) / 0.9),
                       amplitude="magnitude", zero_point=zp)
    model = oracle.render(s0, t)
    rng = np.random.default_rng(5)
    d = model + 0.02 * np.max(model) * rng.standard_normal(model.shape)
    s = oracle.System(20, 18, 0.1, 2, s0.psf, d, np.full(model.shape, 1.0 / (0.02 * np.max(model)) ** 2),
                      amplitude="magnitude", zero_point=zp)
    t[14] += 0.1; t[6] -= 0.05; t[12] += 0.05
    ll, g = oracle.loglike_grad(s, t)
    assert ll == pytest.approx(oracle.loglike(s, t), rel=1e-14)
    fd = np.array([_fd_grad(s, t, k) for k in range(17)])
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd))
    # the amplitude, radius and index entries differ from the intensity form's
    u = t.copy()
    u[5] = oracle.intensity_from_magnitude(t[5], t[6], t[7], zp)
    u[12] = oracle.intensity_from_magnitude(t[12], t[13], t[14], zp)
    si = oracle.System(20, 18, 0.1, 2, s0.psf, d, s.weight.reshape(model.shape))
    _, gi = oracle.loglike_grad(si, u)
    assert g[12] == pytest.approx(gi[12] * u[12] * (-0.4 * math.log(10.0)), rel=1e-10)
    assert g[13] == pytest.approx(gi[13] + gi[12] * u[12] * (-2.0 / t[13]), rel=1e-9)
    k = [0, 1, 2, 3, 4, 8, 9, 10, 11, 15, 16]
    assert np.allclose(g[k], gi[k], rtol=1e-12, atol=1e-12 * np.max(np.abs(gi)))
