"""Pins of the oracle's pixel integration rules (Sec. 3.1 Eq. 14, Sec. 4.5):
Gauss-Legendre against numpy's leggauss, the Kronrod extensions by their
defining exactness (monomials up to degree 3n + 1; the embedded Gauss rule up
to 2n - 1 and not beyond), interlacing, positivity and symmetry, and the
product rules on a pixel integral with a closed form (a Gaussian source
without lens: products of error functions)."""
import math

import numpy as np
import pytest
from scipy import special

import oracle
from oracle import quadrature as qd

from test_oracle_pins import theta_base


@pytest.mark.parametrize("n", [1, 3, 5, 7, 10])
def test_gauss_legendre_matches_numpy(n):
    x, w = qd.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, atol=1e-14) and np.allclose(w, wr, atol=1e-14)


@pytest.mark.parametrize("n", [3, 5, 7])
def test_kronrod_extension_by_its_definition(n):
    x, wk, gw = qd.gauss_kronrod(n)
    assert len(x) == 2 * n + 1
    mono = lambda k: 0.0 if k % 2 else 2.0 / (k + 1)
    for k in range(3 * n + 2):
        assert abs(np.sum(wk * x ** k) - mono(k)) < 1e-14, k
    for k in range(2 * n):
        assert abs(np.sum(gw * x ** k) - mono(k)) < 1e-14, k
    assert abs(np.sum(gw * x ** (2 * n)) - mono(2 * n)) > 1e-6       # the Gauss rule stops at 2n - 1
    assert np.all(wk > 0)
    assert np.allclose(x, -x[::-1], atol=1e-15) and np.allclose(wk, wk[::-1], atol=1e-15)
    xg = x[gw != 0]
    assert np.allclose(xg, qd.gauss_legendre(n)[0], atol=1e-15)
    assert np.array_equal(np.nonzero(gw)[0], np.arange(1, 2 * n + 1, 2))   # Kronrod and Gauss nodes alternate


def test_explicit_midpoint_rule_equals_the_builtin_one():
    t = theta_base(theta_E=1.0, q_L=0.8, phi_L=0.4, x_S=0.05, y_S=0.02, R_S=0.15, n_S=1.5)
    a = oracle.render(oracle.System(12, 14, 0.07, 4, np.ones((1, 1))), t, apply_psf=False)
    b = oracle.render(oracle.System(12, 14, 0.07, 1, np.ones((1, 1)), rule="sub4"), t, apply_psf=False)
    assert np.allclose(a, b, rtol=1e-13, atol=0)


def test_gauss_kronrod_product_rules_against_exact_pixel_integral():
    """Gaussian source (n = 1/2, q = 1) without lens: every rule converges to the
    error-function closed form; g7k15 to ~1e-12 of the peak, each GK rule beats
    sub16, and the embedded-Gauss error map bounds the actual error of the
    Kronrod result."""
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
    e16 = np.max(np.abs(oracle.render(oracle.System(H, W, d, 16, np.ones((1, 1))), t, apply_psf=False) - exact))
    errs = {}
    for rule in ("g3k7", "g5k11", "g7k15"):
        s = oracle.System(H, W, d, 1, np.ones((1, 1)), rule=rule)
        L = oracle.render(s, t, apply_psf=False)
        errs[rule] = np.max(np.abs(L - exact))
        est = oracle.render_error(s, t)
        assert np.all(est >= 0) and np.all(np.abs(L - exact) <= est + 1e-15 * exact.max())
        assert errs[rule] < e16
    assert errs["g7k15"] < 1e-12 * exact.max()
    assert errs["g3k7"] > errs["g5k11"] > errs["g7k15"]
