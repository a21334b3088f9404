"""FP64 CPU oracle for the forward lensing model -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. The product library never calls it and shares no code
with it.

Functions follow Tessore, Bellagamba & Metcalf (MNRAS 2016):
lens equation Sec. 2.1 Eq. (1); surface brightness Eq. (2); pixel luminosity
Eq. (3) by midpoint subsampling (Sec. 3.1 Eq. (14), Sec. 4.5 "subN" rules);
PSF convolution with replicate padding Sec. 3.1 Eq. (15); log-likelihood
Sec. 3.2 Eq. (17); Sersic profile Sec. 4.1 Eqs. (22)-(23), optionally with its
amplitude set by a total magnitude (Sec. 4.1); SIE lens Sec. 4; image-plane
source positions (Sec. 5).
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

NPAR = 17

_lib = None


class LoSystem(ctypes.Structure):
    _fields_ = [
        ("height", ctypes.c_int32), ("width", ctypes.c_int32),
        ("pixscale", ctypes.c_double),
        ("center_x", ctypes.c_double), ("center_y", ctypes.c_double),
        ("nsub", ctypes.c_int32),
        ("psf_h", ctypes.c_int32), ("psf_w", ctypes.c_int32),
        ("psf", ctypes.POINTER(ctypes.c_double)),
        ("data", ctypes.POINTER(ctypes.c_double)),
        ("weight", ctypes.POINTER(ctypes.c_double)),
        ("rule_n", ctypes.c_int32),
        ("rule_x", ctypes.POINTER(ctypes.c_double)),
        ("rule_w", ctypes.POINTER(ctypes.c_double)),
        ("amplitude", ctypes.c_int32),
        ("zero_point", ctypes.c_double),
        ("source_position", ctypes.c_int32),
    ]


class LoModel(ctypes.Structure):
    _fields_ = [("n_sie", ctypes.c_int32), ("shear", ctypes.c_int32), ("n_sersic", ctypes.c_int32),
                ("sky", ctypes.c_int32), ("plane", ctypes.c_int32 * 8), ("n_planes", ctypes.c_int32),
                ("sie_plane", ctypes.c_int32 * 8), ("reserved", ctypes.c_int32),
                ("beta", (ctypes.c_double * 8) * 8)]


class Model:
    """A general model (Sec. 5: several lenses and light components, a flat sky,
    free centres). planes: one entry per Sersic, 'image' (unlensed light),
    'source' (lensed), or the index of the plane the light sits on (0..P, P the
    source plane). Parameters: per SIE (x_c, y_c, theta_E, q, phi); the shear
    (gamma, phi_gamma) if any; per Sersic (x, y, I_e, R_e, n, q, phi); the sky
    surface brightness if any.

    Several lens planes (the extension named in Sec. 6): beta, a P x P array whose entries
    beta[i][j], i < j, are the distance ratios of the multi-plane lens equation,
    and sie_planes, the lens plane of every SIE (default all on plane 0)."""

    def __init__(self, n_sie, planes, shear=True, sky=False, sie_planes=None, beta=None):
        planes = list(planes)
        if not 1 <= len(planes) <= 8 or not 0 <= n_sie <= 8:
            raise ValueError("1..8 Sersic components and 0..8 SIEs")
        n_planes = 1 if beta is None else len(beta)
        codes = [0 if q == "image" else n_planes if q == "source" else int(q) for q in planes]
        pl = (ctypes.c_int32 * 8)(*(codes + [0] * (8 - len(codes))))
        sp = [0] * n_sie if sie_planes is None else [int(k) for k in sie_planes]
        if len(sp) != n_sie:
            raise ValueError("one lens plane per SIE")
        b = ((ctypes.c_double * 8) * 8)()
        if beta is not None:
            beta = np.asarray(beta, np.float64)
            for i in range(n_planes):
                for j in range(n_planes):
                    b[i][j] = beta[i, j]
        self._m = LoModel(int(n_sie), int(bool(shear)), len(planes), int(bool(sky)), pl, n_planes,
                          (ctypes.c_int32 * 8)(*(sp + [0] * (8 - len(sp)))), 0, b)
        self.n_planes = n_planes
        self.n_params = lib().lo_model_nparams(ctypes.byref(self._m))

    @property
    def ptr(self):
        return ctypes.byref(self._m)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        d, i, dp = ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        sp = ctypes.POINTER(LoSystem)
        for name, res, args in [
            ("lo_param_count", i, []),
            ("lo_digamma", d, [d]),
            ("lo_gamma_p", d, [d, d]),
            ("lo_bn", d, [d]),
            ("lo_bn_deriv", d, [d]),
            ("lo_intensity_from_magnitude", d, [d, d, d, d]),
            ("lo_sie_deflection", None, [d, d, d, d, d, dp, dp]),
            ("lo_shear_deflection", None, [d, d, d, d, dp, dp]),
            ("lo_sersic", d, [d] * 9),
            ("lo_surface_brightness", d, [dp, d, d]),
            ("lo_surface_brightness_grad", d, [dp, d, d, dp]),
            ("lo_sum_compensated", d, [dp, ctypes.c_int64]),
            ("lo_render", i, [sp, dp, i, dp]),
            ("lo_render_error", i, [sp, dp, dp, dp]),
            ("lo_psf_convolve", i, [i, i, dp, i, i, dp, dp]),
            ("lo_loglike", d, [sp, dp]),
            ("lo_loglike_grad", d, [sp, dp, dp]),
            ("lo_model_nparams", i, [ctypes.c_void_p]),
            ("lo_render_model", i, [sp, ctypes.c_void_p, dp, i, dp]),
            ("lo_loglike_model", d, [sp, ctypes.c_void_p, dp]),
            ("lo_model_positions", i, [ctypes.c_void_p, dp, d, d, dp, dp]),
        ]:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class System:
    """Host-side description of one observation for the oracle.

    All arrays are converted to float64 copies; values the GPU sees in float32
    should be passed already rounded to float32 so both sides read the same numbers.
    """

    def __init__(self, height, width, pixscale, nsub, psf, data=None, weight=None,
                 center_x=0.0, center_y=0.0, rule=None, amplitude="intensity", zero_point=0.0,
                 source_position="source"):
        """rule: None for the nsub x nsub midpoint rule, or a name accepted by
        oracle.quadrature.pixel_rule ('subN', 'point', 'g3k7', 'g5k11', 'g7k15').
        amplitude: 'intensity' (theta[5], theta[12] are I_e) or 'magnitude'
        (they are total magnitudes with the given zero point, Sec. 4.1).
        source_position: 'source' (theta[10], theta[11] are the source centre) or
        'image' (they are an image-plane point that the lens equation maps to
        the source centre, Sec. 5)."""
        if source_position not in ("source", "image"):
            raise ValueError("source_position must be 'source' or 'image'")
        self.source_position = source_position
        if amplitude not in ("intensity", "magnitude"):
            raise ValueError("amplitude must be 'intensity' or 'magnitude'")
        self.amplitude, self.zero_point = amplitude, float(zero_point)
        self.height, self.width = int(height), int(width)
        self.pixscale = float(pixscale)
        self.center_x, self.center_y = float(center_x), float(center_y)
        self.nsub = int(nsub)
        self.psf = np.ascontiguousarray(np.asarray(psf, dtype=np.float64))
        n = self.height * self.width
        self.data = np.ascontiguousarray(np.zeros(n) if data is None else np.asarray(data, np.float64).reshape(-1))
        self.weight = np.ascontiguousarray(np.ones(n) if weight is None else np.asarray(weight, np.float64).reshape(-1))
        self.rule = rule
        self.rule_x = self.rule_w = self.rule_g = None
        rn, rx, rw = 0, None, None
        if rule is not None:
            from .quadrature import pixel_rule
            x, w, g = pixel_rule(rule)
            self.rule_x, self.rule_w = np.ascontiguousarray(x), np.ascontiguousarray(w)
            self.rule_g = None if g is None else np.ascontiguousarray(g)
            rn, rx, rw = len(x), _dp(self.rule_x), _dp(self.rule_w)
        self._s = LoSystem(self.height, self.width, self.pixscale, self.center_x, self.center_y,
                           self.nsub, self.psf.shape[0], self.psf.shape[1],
                           _dp(self.psf), _dp(self.data), _dp(self.weight), rn, rx, rw,
                           1 if amplitude == "magnitude" else 0, self.zero_point,
                           1 if source_position == "image" else 0)

    @property
    def ptr(self):
        return ctypes.byref(self._s)


def _theta(theta):
    t = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(-1))
    assert t.size == NPAR
    return t


def bn(n):
    """b_n with P(2n, b_n) = 1/2 (half-light normalisation of Eq. 22)."""
    return lib().lo_bn(float(n))


def bn_deriv(n):
    return lib().lo_bn_deriv(float(n))


def intensity_from_magnitude(m, Re, n, zero_point=0.0):
    """I_e of a Sersic component of total magnitude m (Sec. 4.1): total flux
    10^(-0.4 (m - zero_point)) = 2 pi n R_e^2 I_e e^(b_n) Gamma(2n) / b_n^(2n)."""
    return lib().lo_intensity_from_magnitude(float(m), float(Re), float(n), float(zero_point))


def digamma(z):
    return lib().lo_digamma(float(z))


def gamma_p(a, x):
    return lib().lo_gamma_p(float(a), float(x))


def sie_deflection(theta_e, q, phi, x, y):
    ax, ay = ctypes.c_double(), ctypes.c_double()
    lib().lo_sie_deflection(theta_e, q, phi, x, y, ctypes.byref(ax), ctypes.byref(ay))
    return ax.value, ay.value


def shear_deflection(gamma, phi, x, y):
    ax, ay = ctypes.c_double(), ctypes.c_double()
    lib().lo_shear_deflection(gamma, phi, x, y, ctypes.byref(ax), ctypes.byref(ay))
    return ax.value, ay.value


def sersic(x, y, x0, y0, Ie, Re, n, q, phi):
    return lib().lo_sersic(x, y, x0, y0, Ie, Re, n, q, phi)


def surface_brightness(theta, x, y):
    t = _theta(theta)
    return lib().lo_surface_brightness(_dp(t), float(x), float(y))


def surface_brightness_grad(theta, x, y):
    t = _theta(theta)
    g = np.zeros(NPAR)
    v = lib().lo_surface_brightness_grad(_dp(t), float(x), float(y), _dp(g))
    return v, g


def sum_compensated(x):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
    return lib().lo_sum_compensated(_dp(a), a.size)


def render(system, theta, apply_psf=True):
    t = _theta(theta)
    out = np.empty(system.height * system.width)
    rc = lib().lo_render(system.ptr, _dp(t), int(bool(apply_psf)), _dp(out))
    if rc != 0:
        raise ValueError("oracle render: invalid system")
    return out.reshape(system.height, system.width)


def render_error(system, theta):
    """|Kronrod - embedded Gauss| per pixel (before the PSF) for a system built
    with a Gauss-Kronrod rule."""
    if system.rule_g is None:
        raise ValueError("render_error needs a Gauss-Kronrod rule")
    t = _theta(theta)
    out = np.empty(system.height * system.width)
    if lib().lo_render_error(system.ptr, _dp(t), _dp(system.rule_g), _dp(out)) != 0:
        raise ValueError("oracle render_error: invalid system")
    return out.reshape(system.height, system.width)


def psf_convolve(image, psf):
    img = np.ascontiguousarray(np.asarray(image, dtype=np.float64))
    F = np.ascontiguousarray(np.asarray(psf, dtype=np.float64))
    out = np.empty_like(img)
    rc = lib().lo_psf_convolve(img.shape[0], img.shape[1], _dp(img), F.shape[0], F.shape[1], _dp(F), _dp(out))
    if rc != 0:
        raise ValueError("oracle psf_convolve: invalid arguments")
    return out


def loglike(system, theta):
    t = _theta(theta)
    return lib().lo_loglike(system.ptr, _dp(t))


def loglike_grad(system, theta):
    t = _theta(theta)
    g = np.zeros(NPAR)
    v = lib().lo_loglike_grad(system.ptr, _dp(t), _dp(g))
    return v, g


def render_composite(system, thetas, sky=0.0, apply_psf=True):
    """Model image of a composite model (Sec. 5: several light components and a
    flat sky): the sum of the components' pixel luminosities (each a 17-parameter
    point) plus the sky's, sky x pixscale^2 per pixel, then the PSF (Eq. 15)."""
    L = sum(render(system, t, apply_psf=False) for t in np.atleast_2d(thetas))
    L = L + float(sky) * system.pixscale ** 2
    return psf_convolve(L, system.psf) if apply_psf else L


def loglike_composite(system, thetas, sky=0.0):
    """log L (Eq. 17) of a composite model: -1/2 sum_i w_i (d_i - L*_i)^2 with the
    compensated sum."""
    m = render_composite(system, thetas, sky).reshape(-1)
    r = system.data - m
    return -0.5 * sum_compensated(system.weight * r * r)


def loglike_multiband(band_systems, band_thetas, band_skies=None):
    """log L of a simultaneous fit of several bands (Sec. 6 names it as an
    extension): the bands' noise is independent, so the log-likelihoods of the
    bands (Eq. 17, each a composite model on its own system) add."""
    skies = [0.0] * len(band_systems) if band_skies is None else band_skies
    return sum(loglike_composite(s, t, k) for s, t, k in zip(band_systems, band_thetas, skies))


def render_model(system, model, params, apply_psf=True):
    """Image of a general model (Model): Eqs. 1-3 with the model's deflectors and
    light components, Eq. 14 on the system's rule, then Eq. 15."""
    t = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    assert t.size == model.n_params
    out = np.empty(system.height * system.width)
    if lib().lo_render_model(system.ptr, model.ptr, _dp(t), int(bool(apply_psf)), _dp(out)) != 0:
        raise ValueError("oracle render_model: invalid system or model")
    return out.reshape(system.height, system.width)


def model_positions(model, params, x, y):
    """Position of the ray through the image-plane point (x, y) on every plane:
    an array [(x_0, y_0), ..., (x_P, y_P)], lens planes 0..P-1 and the source
    plane P."""
    t = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    assert t.size == model.n_params
    px, py = np.empty(model.n_planes + 1), np.empty(model.n_planes + 1)
    if lib().lo_model_positions(model.ptr, _dp(t), float(x), float(y), _dp(px), _dp(py)) != 0:
        raise ValueError("oracle model_positions: invalid model or parameters")
    return np.stack([px, py], axis=1)


def loglike_model(system, model, params):
    t = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    assert t.size == model.n_params
    return lib().lo_loglike_model(system.ptr, model.ptr, _dp(t))
