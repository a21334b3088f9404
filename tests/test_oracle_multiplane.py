"""Pins of the oracle's multi-plane lensing (the extension named in Sec. 6, in
the standard form of the multi-plane lens equation): closed forms for singular
isothermal spheres on an axis (whose deflection has the constant length
theta_E), the two limits of the distance ratio (0: the planes coincide and the
deflections add; 1: the second plane sits at the source of the first, so the
two lens maps compose), and light on an intermediate plane in those limits."""
import math

import numpy as np
import pytest

import oracle

from test_oracle_model import system


def sis(xc, yc, te):
    """An isothermal sphere (q = 1) of Einstein radius te centred at (xc, yc)."""
    return [xc, yc, te, 1.0, 0.0]


def source(x=0.1, y=-0.05):
    return [x, y, 1.0, 0.3, 1.5, 0.7, 0.4]


def test_two_spheres_on_an_axis():
    """On the x axis: x_1 = x - b01 te0 sign(x), x_2 = x - te0 sign(x) - te1 sign(x_1 - c1)."""
    te0, te1, c1, b01 = 1.1, 0.4, 0.25, 0.63
    m = oracle.Model(2, ["source"], shear=False, sie_planes=[0, 1], beta=[[0, b01], [0, 0]])
    p = sis(0, 0, te0) + sis(c1, 0, te1) + source()
    for x in (2.3, 1.0, 0.6, -0.2, -1.7):
        pos = oracle.model_positions(m, p, x, 0.0)
        x1 = x - b01 * te0 * math.copysign(1, x)
        x2 = x - te0 * math.copysign(1, x) - te1 * math.copysign(1, x1 - c1)
        assert pos[0] == pytest.approx([x, 0.0], abs=1e-15)
        assert pos[1] == pytest.approx([x1, 0.0], abs=1e-14)
        assert pos[2] == pytest.approx([x2, 0.0], abs=1e-14)


def test_three_planes_use_each_distance_ratio_once():
    """Three spheres on the axis with distinct ratios b01, b02, b12: a transposed
    or misplaced ratio changes x_2."""
    te, c = [0.9, 0.5, 0.3], [0.0, 0.2, -0.1]
    b01, b02, b12 = 0.55, 0.8, 0.35
    beta = np.zeros((3, 3))
    beta[0, 1], beta[0, 2], beta[1, 2] = b01, b02, b12
    m = oracle.Model(3, ["source"], shear=False, sie_planes=[0, 1, 2], beta=beta)
    p = sis(c[0], 0, te[0]) + sis(c[1], 0, te[1]) + sis(c[2], 0, te[2]) + source()
    sg = lambda v: math.copysign(1, v)
    for x in (2.0, 1.3, -1.4):
        a0 = te[0] * sg(x - c[0])
        x1 = x - b01 * a0
        a1 = te[1] * sg(x1 - c[1])
        x2 = x - b02 * a0 - b12 * a1
        a2 = te[2] * sg(x2 - c[2])
        x3 = x - a0 - a1 - a2
        pos = oracle.model_positions(m, p, x, 0.0)
        assert pos[:, 0] == pytest.approx([x, x1, x2, x3], abs=1e-14)
        assert np.all(np.abs(pos[:, 1]) <= 1e-15)


def test_a_sphere_off_the_axis_of_the_ray():
    """A sphere at plane 1 deflects the ray towards its centre by te along the
    unit vector from the centre to x_1 (any direction, not only on an axis)."""
    b01 = 0.4
    m = oracle.Model(2, ["source"], shear=False, sie_planes=[0, 1], beta=[[0, b01], [0, 0]])
    p = sis(0.1, -0.2, 0.8) + sis(-0.3, 0.5, 0.35) + source()
    for x, y in [(1.2, 0.7), (-0.9, 1.4), (0.2, -1.3)]:
        d0 = np.array([x - 0.1, y + 0.2])
        a0 = 0.8 * d0 / np.linalg.norm(d0)
        x1 = np.array([x, y]) - b01 * a0
        d1 = x1 - np.array([-0.3, 0.5])
        a1 = 0.35 * d1 / np.linalg.norm(d1)
        pos = oracle.model_positions(m, p, x, y)
        assert np.allclose(pos[1], x1, rtol=0, atol=1e-14)
        assert np.allclose(pos[2], np.array([x, y]) - a0 - a1, rtol=0, atol=1e-14)


# Two elliptical lenses with a shear (on plane 0) and a source, as one plane
# (deflections added) and as two planes.
LENSES = [0.02, -0.03, 1.05, 0.72, 0.4] + [0.55, 0.35, 0.25, 0.8, 1.9]
SHEAR = [0.05, 0.6]
SRC = [0.08, -0.04, 1.2, 0.25, 1.3, 0.65, 2.2]
HOST = [0.02, -0.03, 0.6, 0.9, 3.5, 0.8, 0.4]
COMPANION = [0.55, 0.35, 0.3, 0.3, 2.0, 0.7, 1.1]


def two_plane(b01, planes):
    return oracle.Model(2, planes, shear=True, sie_planes=[0, 1], beta=[[0, b01], [0, 0]])


def test_coincident_planes_add_the_deflections():
    """beta = 0: x_1 = x, and the source position is x - alpha_0(x) - alpha_1(x),
    the one-plane model with both lenses; light on plane 1 is light at x."""
    s = system()
    p = np.array(LENSES + SHEAR + HOST + COMPANION + SRC)
    one = oracle.Model(2, ["image", "image", "source"], shear=True)
    two = two_plane(0.0, [0, 1, 2])
    assert np.allclose(oracle.render_model(s, two, p), oracle.render_model(s, one, p), rtol=1e-13, atol=0)


def test_a_plane_at_the_source_of_the_first_composes_the_lens_maps():
    """beta = 1: x_1 is the first lens's source-plane position and x_2 the second
    lens's map applied to it; light on plane 1 is the first lens's lensed light."""
    p = np.array(LENSES + SHEAR + SRC)
    two = two_plane(1.0, ["source"])
    first = oracle.Model(1, ["source"], shear=True)
    second = oracle.Model(1, ["source"], shear=False)
    pf = np.array(LENSES[:5] + SHEAR + SRC)
    ps = np.array(LENSES[5:] + SRC)
    for x, y in [(0.9, 0.3), (-0.4, 1.1), (0.05, -0.7), (1.6, -1.2)]:
        pos = oracle.model_positions(two, p, x, y)
        b1 = oracle.model_positions(first, pf, x, y)[1]
        b2 = oracle.model_positions(second, ps, *b1)[1]
        assert np.allclose(pos[1], b1, rtol=0, atol=1e-14)
        assert np.allclose(pos[2], b2, rtol=0, atol=1e-14)
    s = system()
    mid = two_plane(1.0, [1])
    lensed_once = oracle.Model(1, ["source"], shear=True)
    a = oracle.render_model(s, mid, np.array(LENSES + SHEAR + SRC))
    b = oracle.render_model(s, lensed_once, pf)
    assert np.allclose(a, b, rtol=1e-13, atol=0)


def test_one_plane_is_the_single_plane_model():
    """P = 1 with explicit (ignored) ratios is the general model of one plane."""
    s = system()
    p = np.array(LENSES + SHEAR + HOST + SRC)
    a = oracle.render_model(s, oracle.Model(2, ["image", "source"], shear=True), p)
    b = oracle.render_model(s, oracle.Model(2, [0, 1], shear=True, sie_planes=[0, 0], beta=[[0.0]]), p)
    assert np.array_equal(a, b)


def test_invalid_plane_layouts():
    p = np.array(LENSES + SHEAR + SRC)
    s = system()
    for kw in [dict(sie_planes=[0, 2], beta=[[0, 0.5], [0, 0]]),        # SIE on no lens plane
               dict(sie_planes=[0, 1], beta=[[0, 1.5], [0, 0]]),        # ratio above 1
               dict(sie_planes=[0, 1], beta=[[0, -0.1], [0, 0]])]:      # ratio below 0
        m = oracle.Model(2, ["source"], shear=True, **kw)
        assert np.all(np.isnan(oracle.render_model(s, m, p)))
    m = oracle.Model(2, [3], shear=True, sie_planes=[0, 1], beta=[[0, 0.5], [0, 0]])   # light beyond the source
    assert np.all(np.isnan(oracle.render_model(s, m, p)))
