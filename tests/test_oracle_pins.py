"""Pins of the FP64 oracle against closed forms, invariants, library routines and
brute force -- none of which reuse the oracle's own formulas.

Paper: Tessore, Bellagamba & Metcalf, LENSED (MNRAS 2016). Citations name the
section and equation each pinned step follows.
"""
import math

import numpy as np
import pytest
from scipy import integrate, ndimage, special

import oracle

RNG = np.random.default_rng(20160101)


def theta_base(**kw):
    """A parameter vector with no lens, no shear and no lens light, overridden by kw."""
    names = ["theta_E", "q_L", "phi_L", "gamma", "phi_gamma", "I_H", "R_H", "n_H", "q_H", "phi_H",
             "x_S", "y_S", "I_S", "R_S", "n_S", "q_S", "phi_S"]
    t = dict(theta_E=0.0, q_L=1.0, phi_L=0.0, gamma=0.0, phi_gamma=0.0, I_H=0.0, R_H=1.0, n_H=1.0,
             q_H=1.0, phi_H=0.0, x_S=0.0, y_S=0.0, I_S=1.0, R_S=0.2, n_S=1.0, q_S=1.0, phi_S=0.0)
    t.update(kw)
    return np.array([t[k] for k in names], dtype=np.float64)


# ---------------------------------------------------------------------------
# Sersic normalisation b_n (Sec. 4.1, Eq. 22: R_e is the half-light radius)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,expected", [
    (0.5, math.log(2.0)),            # Gaussian case: closed form ln 2
    (1.0, 1.678346990017), (2.0, 3.672060748851), (4.0, 7.669249442501),
    (6.0, 11.668363153045), (8.0, 15.667929544317)])
def test_bn_values(n, expected):
    assert oracle.bn(n) == pytest.approx(expected, rel=2e-12)


def test_bn_matches_library_inverse():
    for n in RNG.uniform(0.2, 10.0, size=25):
        assert oracle.bn(n) == pytest.approx(special.gammaincinv(2 * n, 0.5), rel=1e-11)


def test_gamma_p_and_digamma_match_library():
    for a, x in zip(RNG.uniform(0.4, 20, 30), RNG.uniform(0.01, 25, 30)):
        assert oracle.gamma_p(a, x) == pytest.approx(special.gammainc(a, x), rel=1e-12, abs=1e-300)
    for z in RNG.uniform(0.05, 40, 30):
        assert oracle.digamma(z) == pytest.approx(special.digamma(z), rel=1e-12, abs=1e-13)


def test_bn_derivative_against_richardson_fd_of_library_root():
    def b(n):
        return special.gammaincinv(2 * n, 0.5)
    for n in [0.3, 0.5, 1.0, 1.7, 3.0, 6.0, 9.5]:
        h = 1e-3 * n
        d1 = (b(n + h) - b(n - h)) / (2 * h)
        d2 = (b(n + h / 2) - b(n - h / 2)) / h
        rich = (4 * d2 - d1) / 3
        assert oracle.bn_deriv(n) == pytest.approx(rich, rel=1e-8)


def test_half_light_radius_by_quadrature():
    """Enclosed flux at R_e is half the total (radial quadrature of the oracle's profile)."""
    for n in [0.5, 1.0, 2.5, 4.0]:
        Re = 0.3
        f = lambda r: 2 * math.pi * r * oracle.sersic(r, 0.0, 0.0, 0.0, 1.0, Re, n, 1.0, 0.0)
        inner = integrate.quad(f, 0, Re, limit=200, epsabs=0, epsrel=1e-12)[0]
        total = inner + integrate.quad(f, Re, np.inf, limit=400, epsabs=0, epsrel=1e-12)[0]
        assert inner / total == pytest.approx(0.5, rel=1e-8)


def test_sersic_special_cases_gaussian_and_exponential():
    Re, Ie = 0.25, 1.7
    for r in [0.0, 0.05, 0.25, 0.6, 1.3]:
        g = 2 * Ie * math.exp(-math.log(2) * r * r / (Re * Re))      # n = 1/2
        assert oracle.sersic(r, 0, 0, 0, Ie, Re, 0.5, 1.0, 0.0) == pytest.approx(g, rel=1e-13)
        b1 = special.gammaincinv(2.0, 0.5)
        e = Ie * math.exp(-b1 * (r / Re - 1))                       # n = 1
        assert oracle.sersic(0, r, 0, 0, Ie, Re, 1.0, 1.0, 0.0) == pytest.approx(e, rel=1e-11)


def test_sersic_position_angle_and_radius_convention():
    """The major axis points at phi counter-clockwise from +x (Sec. 4); R is the
    geometric-mean radius sqrt(q x'^2 + y'^2/q) (Eq. 23)."""
    q, phi, Re, n = 0.5, 0.6, 0.3, 1.0
    d = 0.4
    major = (d * math.cos(phi), d * math.sin(phi))
    minor = (-d * math.sin(phi), d * math.cos(phi))
    Imaj = oracle.sersic(*major, 0, 0, 1.0, Re, n, q, phi)
    Imin = oracle.sersic(*minor, 0, 0, 1.0, Re, n, q, phi)
    assert Imaj > Imin
    b = special.gammaincinv(2 * n, 0.5)
    assert Imaj == pytest.approx(math.exp(-b * (math.sqrt(q) * d / Re - 1)), rel=1e-12)
    assert Imin == pytest.approx(math.exp(-b * (d / math.sqrt(q) / Re - 1)), rel=1e-12)


# ---------------------------------------------------------------------------
# Lens models (Sec. 2.1 Eq. 1; SIE of Sec. 4; external shear of Sec. 5)
# ---------------------------------------------------------------------------

def test_sis_closed_form():
    te = 1.3
    for x, y in RNG.uniform(-3, 3, size=(20, 2)):
        ax, ay = oracle.sie_deflection(te, 1.0, RNG.uniform(0, math.pi), x, y)
        r = math.hypot(x, y)
        assert ax == pytest.approx(te * x / r, rel=1e-13, abs=1e-15)
        assert ay == pytest.approx(te * y / r, rel=1e-13, abs=1e-15)


def test_sie_continuous_at_q_one_and_at_series_switch():
    te, phi = 1.1, 0.7
    for x, y in RNG.uniform(-2, 2, size=(10, 2)):
        a1 = np.array(oracle.sie_deflection(te, 1.0, phi, x, y))
        a2 = np.array(oracle.sie_deflection(te, 1.0 - 1e-9, phi, x, y))
        assert np.max(np.abs(a1 - a2)) < 1e-8
        qs = math.sqrt(1.0 - 1e-4)          # series / closed-form switch at 1 - q^2 = 1e-4
        lo = np.array(oracle.sie_deflection(te, qs * (1 + 1e-12), phi, x, y))
        hi = np.array(oracle.sie_deflection(te, qs * (1 - 1e-12), phi, x, y))
        assert np.max(np.abs(lo - hi)) < 1e-12


def _sie_fd(te, q, phi, x, y, h=1e-5):
    axp, ayp = oracle.sie_deflection(te, q, phi, x + h, y)
    axm, aym = oracle.sie_deflection(te, q, phi, x - h, y)
    bxp, byp = oracle.sie_deflection(te, q, phi, x, y + h)
    bxm, bym = oracle.sie_deflection(te, q, phi, x, y - h)
    div = (axp - axm) / (2 * h) + (byp - bym) / (2 * h)
    curl = (ayp - aym) / (2 * h) - (bxp - bxm) / (2 * h)
    return div, curl


def test_sie_divergence_is_twice_convergence_and_curl_free():
    for _ in range(20):
        te, q, phi = RNG.uniform(0.5, 2), RNG.uniform(0.3, 0.98), RNG.uniform(0, math.pi)
        x, y = RNG.uniform(-2, 2, size=2)
        c, s = math.cos(phi), math.sin(phi)
        xp, yp = c * x + s * y, -s * x + c * y
        kappa = te / (2 * math.sqrt(q * xp * xp + yp * yp / q))
        div, curl = _sie_fd(te, q, phi, x, y)
        assert div == pytest.approx(2 * kappa, rel=1e-7)
        assert abs(curl) < 1e-7 * kappa


def test_sie_flux_through_critical_ellipse():
    """Gauss: the outward flux of alpha through q x'^2 + y'^2/q = theta_E^2 is
    2 * (enclosed mass) = 2 pi theta_E^2, so theta_E is the equivalent circular
    Einstein radius."""
    te, q, phi = 1.25, 0.55, 0.4
    c, s = math.cos(phi), math.sin(phi)
    a_, b_ = te / math.sqrt(q), te * math.sqrt(q)      # semi-axes along x', y'

    def integrand(t):
        xp, yp = a_ * math.cos(t), b_ * math.sin(t)
        nx_p, ny_p = b_ * math.cos(t), a_ * math.sin(t)   # outward normal * dl/dt
        x, y = c * xp - s * yp, s * xp + c * yp
        nx, ny = c * nx_p - s * ny_p, s * nx_p + c * ny_p
        ax, ay = oracle.sie_deflection(te, q, phi, x, y)
        return ax * nx + ay * ny

    flux = integrate.quad(integrand, 0, 2 * math.pi, limit=200, epsabs=0, epsrel=1e-12)[0]
    assert flux == pytest.approx(2 * math.pi * te * te, rel=1e-10)


def test_sie_rotation_covariance():
    te, q = 0.9, 0.6
    for phi in [0.3, 1.2, 2.9]:
        for x, y in RNG.uniform(-2, 2, size=(5, 2)):
            c, s = math.cos(phi), math.sin(phi)
            ax0, ay0 = oracle.sie_deflection(te, q, 0.0, x, y)
            ax, ay = oracle.sie_deflection(te, q, phi, c * x - s * y, s * x + c * y)
            assert ax == pytest.approx(c * ax0 - s * ay0, abs=1e-13)
            assert ay == pytest.approx(s * ax0 + c * ay0, abs=1e-13)


def test_shear_is_gradient_of_its_potential():
    """alpha_gamma = grad of psi = (g1 (x^2 - y^2))/2 + g2 x y, with g1 = g cos 2phi,
    g2 = g sin 2phi; the stretch of images is along phi."""
    g, phi = 0.07, 0.35
    g1, g2 = g * math.cos(2 * phi), g * math.sin(2 * phi)
    pot = lambda x, y: 0.5 * g1 * (x * x - y * y) + g2 * x * y
    h = 1e-5
    for x, y in RNG.uniform(-2, 2, size=(8, 2)):
        ax, ay = oracle.shear_deflection(g, phi, x, y)
        assert ax == pytest.approx((pot(x + h, y) - pot(x - h, y)) / (2 * h), abs=1e-10)
        assert ay == pytest.approx((pot(x, y + h) - pot(x, y - h)) / (2 * h), abs=1e-10)
    # Along phi the lens equation contracts (beta = (1 - g) x): images are stretched there.
    ax, ay = oracle.shear_deflection(g, phi, math.cos(phi), math.sin(phi))
    assert ax == pytest.approx(g * math.cos(phi), abs=1e-14)
    assert ay == pytest.approx(g * math.sin(phi), abs=1e-14)


def test_no_lens_identity_map():
    t = theta_base(x_S=0.13, y_S=-0.21, R_S=0.3, n_S=2.2, q_S=0.6, phi_S=0.8, I_S=1.4)
    for x, y in RNG.uniform(-1, 1, size=(10, 2)):
        assert oracle.surface_brightness(t, x, y) == pytest.approx(
            oracle.sersic(x, y, 0.13, -0.21, 1.4, 0.3, 2.2, 0.6, 0.8), rel=1e-14)


def test_surface_brightness_conservation_sis():
    """SIS: the centre of a source at beta_0 (|beta_0| < theta_E) is imaged at
    x = (|beta_0| +- theta_E) beta_0/|beta_0|, where the lensed surface brightness
    equals the source's central value I_e e^{b_n}."""
    te, bx, by, n, Ie = 1.0, 0.17, -0.08, 1.5, 0.9
    t = theta_base(theta_E=te, x_S=bx, y_S=by, n_S=n, I_S=Ie, R_S=0.2, q_S=0.7, phi_S=0.4)
    b = np.hypot(bx, by)
    peak = Ie * math.exp(special.gammaincinv(2 * n, 0.5))
    for sgn in (+1, -1):
        x = (b + sgn * te) * bx / b
        y = (b + sgn * te) * by / b
        assert oracle.surface_brightness(t, x, y) == pytest.approx(peak, rel=1e-9)
    # nowhere brighter than the source's maximum
    for x, y in RNG.uniform(-2, 2, size=(200, 2)):
        assert oracle.surface_brightness(t, x, y) <= peak * (1 + 1e-12)


def test_point_probe_of_renderer_is_surface_brightness():
    """A 1x1 image with the point rule samples the surface brightness at its centre."""
    t = theta_base(theta_E=1.1, q_L=0.7, phi_L=0.3, gamma=0.04, phi_gamma=1.0, I_H=0.1, R_H=1.2,
                   n_H=3.0, q_H=0.8, phi_H=0.2, x_S=0.05, y_S=0.02, n_S=1.2, q_S=0.8, phi_S=0.5)
    for x, y in RNG.uniform(-2, 2, size=(5, 2)):
        sysm = oracle.System(1, 1, 0.05, 1, np.ones((1, 1)), center_x=x, center_y=y)
        L = oracle.render(sysm, t, apply_psf=False)
        assert L[0, 0] == pytest.approx(oracle.surface_brightness(t, x, y) * 0.05 ** 2, rel=1e-14)


# ---------------------------------------------------------------------------
# Pixel integration (Eq. 3 by the N x N midpoint rule of Eq. 14)
# ---------------------------------------------------------------------------

def test_sersic_total_flux_closed_form():
    """Sum of pixel luminosities -> 2 pi n R_e^2 I_e e^{b_n} b_n^{-2n} Gamma(2n),
    independent of q because R is area preserving (Eq. 23). The midpoint error
    at the central cusp shrinks faster than 1/N^2."""
    for n, q, phi, tol in [(0.5, 0.6, 0.4, 1e-12), (1.0, 0.8, 1.1, 5e-6), (1.5, 0.5, 2.0, 5e-5),
                           (2.0, 0.7, 0.3, 3e-4)]:
        Re, Ie = 0.1, 1.3
        t = theta_base(x_S=0.0, y_S=0.0, I_S=Ie, R_S=Re, n_S=n, q_S=q, phi_S=phi)
        b = special.gammaincinv(2 * n, 0.5)
        F = 2 * math.pi * n * Re * Re * Ie * math.exp(b) * b ** (-2 * n) * special.gamma(2 * n)
        err = []
        for N in (4, 8):
            sysm = oracle.System(200, 200, 0.03, N, np.ones((1, 1)))
            err.append(abs(oracle.render(sysm, t, apply_psf=False).sum() / F - 1))
        assert err[1] < tol
        assert err[1] < err[0] / 4 or err[0] < 1e-12


def test_midpoint_rule_against_exact_pixel_integral_of_gaussian():
    """n = 1/2, q = 1 source without lens: the pixel integral has a closed form
    in error functions; the N x N midpoint error falls as 1/N^2."""
    Re, Ie = 0.08, 1.0
    a = math.log(2) / (Re * Re)
    t = theta_base(x_S=0.013, y_S=-0.021, I_S=Ie, R_S=Re, n_S=0.5)
    H = W = 16
    d = 0.05
    xe = (np.arange(W + 1) - W / 2) * d
    ye = (np.arange(H + 1) - H / 2) * d
    ex = special.erf(math.sqrt(a) * (xe - 0.013))
    ey = special.erf(math.sqrt(a) * (ye + 0.021))
    exact = 2 * Ie * (math.pi / (4 * a)) * np.outer(np.diff(ey), np.diff(ex))
    errs = []
    for N in (2, 4, 8, 16):
        L = oracle.render(oracle.System(H, W, d, N, np.ones((1, 1))), t, apply_psf=False)
        errs.append(np.max(np.abs(L - exact)))
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.5 < e1 / e2 < 4.5
    assert errs[-1] < 1e-3 * exact.max()


def test_magnification_sum_rule_sis():
    """SIS, compact source at |beta| < theta_E: the total flux tends to
    (2 theta_E/|beta|) times the unlensed flux."""
    te, bx, by, Re, n = 1.0, 0.28, 0.11, 0.012, 1.0
    t = theta_base(theta_E=te, x_S=bx, y_S=by, R_S=Re, n_S=n)
    sysm = oracle.System(160, 160, 0.02, 6, np.ones((1, 1)))
    tot = oracle.render(sysm, t, apply_psf=False).sum()
    b = special.gammaincinv(2 * n, 0.5)
    F = 2 * math.pi * n * Re * Re * math.exp(b) * b ** (-2 * n) * special.gamma(2 * n)
    assert tot / F == pytest.approx(2 * te / math.hypot(bx, by), rel=1e-2)


def test_image_rotates_with_model():
    """Rotating every angle and the source position by 90 degrees rotates the image on a
    square grid centred on the lens (checks the transposition of rows and columns)."""
    t = theta_base(theta_E=1.0, q_L=0.7, phi_L=0.3, gamma=0.05, phi_gamma=0.9, I_H=0.2, R_H=0.8,
                   n_H=2.0, q_H=0.8, phi_H=1.1, x_S=0.12, y_S=-0.07, R_S=0.15, n_S=1.3, q_S=0.6, phi_S=0.4)
    r = t.copy()
    for k in (2, 4, 9, 16):
        r[k] += math.pi / 2
    r[10], r[11] = -t[11], t[10]
    F = np.array([[0.0, 1, 0], [1, 4, 1], [0, 1, 0]])
    sysm = oracle.System(24, 24, 0.1, 3, F)
    A = oracle.render(sysm, t)
    B = oracle.render(sysm, r)
    # (x, y) -> (-y, x): pixel (row i, col j) -> (row j, col W-1-i)
    assert np.allclose(B, _rot(A), rtol=1e-11, atol=1e-15)
    assert not np.allclose(B, A, rtol=1e-3)


def _rot(A):
    H, W = A.shape
    B = np.empty_like(A)
    for i in range(H):
        for j in range(W):
            B[j, W - 1 - i] = A[i, j]
    return B


# ---------------------------------------------------------------------------
# PSF convolution (Sec. 3.1, Eq. 15)
# ---------------------------------------------------------------------------

def test_psf_matches_library_convolution_with_nearest_padding():
    """scipy.ndimage.convolve with mode='nearest' is Eq. 15 with replicate padding."""
    img = RNG.random((23, 17))
    for shape in [(3, 3), (5, 7), (1, 9), (7, 1)]:
        F = RNG.random(shape)
        ref = ndimage.convolve(img, F / F.sum(), mode="nearest")
        assert np.allclose(oracle.psf_convolve(img, F), ref, rtol=1e-13, atol=1e-15)


def test_psf_brute_force_asymmetric_3x3():
    img = RNG.random((5, 5))
    F = np.arange(1.0, 10.0).reshape(3, 3)
    Fn = F / F.sum()
    out = np.zeros_like(img)
    for i in range(5):
        for j in range(5):
            for k in (-1, 0, 1):
                for l in (-1, 0, 1):
                    out[i, j] += Fn[1 - k, 1 - l] * img[min(max(i + k, 0), 4), min(max(j + l, 0), 4)]
    assert np.allclose(oracle.psf_convolve(img, F), out, rtol=1e-14)


def test_psf_delta_identity_shift_and_constant():
    img = RNG.random((9, 11))
    d = np.zeros((5, 5)); d[2, 2] = 3.0
    assert np.array_equal(oracle.psf_convolve(img, d), img)
    s = np.zeros((3, 3)); s[2, 1] = 1.0          # offset (+1 row, 0 col)
    out = oracle.psf_convolve(img, s)
    assert np.array_equal(out[1:], img[:-1])      # features move to larger row index (+y)
    assert np.array_equal(out[0], img[0])         # replicate padding at the border
    const = np.full((8, 8), 2.5)
    assert np.allclose(oracle.psf_convolve(const, RNG.random((7, 5))), 2.5, rtol=1e-14)


def test_psf_conserves_flux_when_border_is_empty():
    img = np.zeros((30, 30)); img[8:22, 6:24] = RNG.random((14, 18))
    F = RNG.random((7, 7))
    assert oracle.psf_convolve(img, F).sum() == pytest.approx(img.sum(), rel=1e-13)


def test_separable_gaussian_psf_equals_two_1d_passes():
    img = RNG.random((20, 20))
    g = np.exp(-0.5 * (np.arange(-3, 4) / 1.2) ** 2)
    F = np.outer(g, g)
    two = ndimage.convolve1d(ndimage.convolve1d(img, g / g.sum(), axis=0, mode="nearest"),
                             g / g.sum(), axis=1, mode="nearest")
    assert np.allclose(oracle.psf_convolve(img, F)[3:-3, 3:-3], two[3:-3, 3:-3], rtol=1e-13)


# ---------------------------------------------------------------------------
# Likelihood (Sec. 3.2, Eq. 17)
# ---------------------------------------------------------------------------

def _small_system(data=None, weight=None, N=2, H=20, W=18):
    F = np.exp(-0.5 * ((np.arange(5) - 2)[:, None] ** 2 + (np.arange(5) - 2)[None, :] ** 2) / 0.9)
    return oracle.System(H, W, 0.1, N, F, data, weight)


T_SMALL = theta_base(theta_E=0.8, q_L=0.75, phi_L=0.5, gamma=0.03, phi_gamma=0.4, I_H=0.05, R_H=0.7,
                     n_H=2.5, q_H=0.8, phi_H=0.3, x_S=0.05, y_S=-0.04, I_S=1.2, R_S=0.2, n_S=1.1,
                     q_S=0.7, phi_S=0.9)


def test_chi2_zero_when_model_equals_data():
    model = oracle.render(_small_system(), T_SMALL)
    s = _small_system(data=model, weight=RNG.uniform(0.5, 2, model.size))
    assert oracle.loglike(s, T_SMALL) == 0.0


def test_masked_pixels_do_not_matter_and_constant_sigma():
    model = oracle.render(_small_system(), T_SMALL)
    d = model + 0.01 * RNG.standard_normal(model.shape)
    w = np.full(model.shape, 1.0 / 0.01 ** 2)
    mask = RNG.random(model.shape) < 0.3
    w[mask] = 0.0
    ll = oracle.loglike(_small_system(d, w), T_SMALL)
    d2 = d.copy(); d2[mask] = 1e6 * RNG.standard_normal(mask.sum())
    assert oracle.loglike(_small_system(d2, w), T_SMALL) == ll
    expect = -0.5 * math.fsum((((d - model) ** 2) / 0.01 ** 2)[~mask])
    assert ll == pytest.approx(expect, rel=1e-14)


def test_compensated_sum_equals_fsum():
    for _ in range(5):
        x = RNG.standard_normal(10000) * 10.0 ** RNG.uniform(-8, 8, 10000)
        assert oracle.sum_compensated(x) == pytest.approx(math.fsum(x), rel=2e-16, abs=0)


# ---------------------------------------------------------------------------
# Gradient (derivative of Eq. 17 through Eqs. 1-3, 15)
# ---------------------------------------------------------------------------

def _fd_grad(s, t, k, rel=1e-4):
    h = rel * max(abs(t[k]), 0.05)
    def f(dh):
        u = t.copy(); u[k] += dh
        return oracle.loglike(s, u)
    d1 = (f(h) - f(-h)) / (2 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4 * d2 - d1) / 3


def test_gradient_matches_richardson_finite_differences():
    model = oracle.render(_small_system(), T_SMALL)
    rng = np.random.default_rng(7)
    d = model + 0.003 * rng.standard_normal(model.shape)
    s = _small_system(d, np.full(model.shape, 1e4))
    t = T_SMALL.copy(); t[0] += 0.01; t[14] += 0.05; t[6] -= 0.03
    ll, g = oracle.loglike_grad(s, t)
    assert ll == pytest.approx(oracle.loglike(s, t), rel=1e-14)
    fd = np.array([_fd_grad(s, t, k) for k in range(17)])
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_gradient_special_zeros():
    s = _small_system(RNG.random(20 * 18), np.ones(20 * 18))
    t = T_SMALL.copy(); t[3] = 0.0          # gamma = 0: phi_gamma has no effect
    _, g = oracle.loglike_grad(s, t)
    assert g[4] == 0.0
    t = T_SMALL.copy(); t[15] = 1.0         # circular source: phi_S has no effect
    _, g = oracle.loglike_grad(s, t)
    assert abs(g[16]) < 1e-12 * np.max(np.abs(g))


def test_surface_brightness_gradient_matches_fd():
    t = T_SMALL.copy()
    for x, y in [(0.3, 0.9), (-0.8, 0.2), (0.5, -0.6)]:
        v, g = oracle.surface_brightness_grad(t, x, y)
        for k in range(17):
            h = 1e-5 * max(abs(t[k]), 0.1)
            u, w = t.copy(), t.copy(); u[k] += h; w[k] -= h
            fd = (oracle.surface_brightness(u, x, y) - oracle.surface_brightness(w, x, y)) / (2 * h)
            assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-8 * max(1.0, abs(v)))


def test_invalid_parameters_give_nan():
    s = _small_system(RNG.random(20 * 18), np.ones(20 * 18))
    for k, bad in [(1, 0.0), (1, 1.2), (13, -0.1), (14, 0.0), (8, float("nan"))]:
        t = T_SMALL.copy(); t[k] = bad
        assert math.isnan(oracle.loglike(s, t))
