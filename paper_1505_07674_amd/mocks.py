"""Seeded synthetic inputs for the forward lensing likelihood.

This module holds no part of the method's arithmetic: it only draws parameter
points from priors, samples PSF shapes on the pixel grid, builds masks and
noise, and assembles a mock observation from a noiseless model image that the
caller supplies (rendered by whichever implementation the caller trusts).

The workloads stand in for the paper's HST-like mocks and SLACS cutouts, which
are not available: 0.05"/px pixels and cutouts bracketing 120x120 (Sec. 4),
an F814W-like 0.1" PSF in place of TinyTim (Sec. 4), an SIE at the image
centre (Sec. 4) and Sersic ranges overlapping those of Sec. 4.1 and Sec. 4.

Parameter layout (17 values, lens at the coordinate origin):
  0 theta_E  1 q_L  2 phi_L  3 gamma  4 phi_gamma
  5 I_H  6 R_H  7 n_H  8 q_H  9 phi_H
 10 x_S 11 y_S 12 I_S 13 R_S 14 n_S 15 q_S 16 phi_S
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

NPAR = 17
PARAM_NAMES = [
    "theta_E", "q_L", "phi_L", "gamma", "phi_gamma",
    "I_H", "R_H", "n_H", "q_H", "phi_H",
    "x_S", "y_S", "I_S", "R_S", "n_S", "q_S", "phi_S",
]
PIXSCALE = 0.05  # arcsec per pixel (Sec. 4)


@dataclass
class Prior:
    """Independent uniform priors; parameters with low == high are fixed."""
    low: np.ndarray
    high: np.ndarray

    @property
    def free(self) -> np.ndarray:
        return np.nonzero(self.high > self.low)[0]

    def from_unit(self, u: np.ndarray) -> np.ndarray:
        """Map points of the unit cube (shape [..., 17]) onto the prior box."""
        return self.low + np.asarray(u) * (self.high - self.low)

    def to_unit(self, theta: np.ndarray) -> np.ndarray:
        w = np.where(self.high > self.low, self.high - self.low, 1.0)
        return (np.asarray(theta) - self.low) / w

    def sample(self, n: int, seed: int) -> np.ndarray:
        rng = np.random.default_rng(seed)
        u = rng.random((n, NPAR))
        return self.from_unit(u).astype(np.float32)


def _prior(spec: Dict[int, Tuple[float, float]], fixed: np.ndarray) -> Prior:
    lo = np.array(fixed, dtype=np.float64)
    hi = np.array(fixed, dtype=np.float64)
    for k, (a, b) in spec.items():
        lo[k], hi[k] = a, b
    return Prior(lo, hi)


# ---------------------------------------------------------------------------
# PSF shapes, sampled at pixel-centre offsets (not normalised: the library and
# the oracle normalise the array themselves, Sec. 3.1).
# ---------------------------------------------------------------------------

def gaussian_psf(size: int, fwhm_arcsec: float, pixscale: float = PIXSCALE) -> np.ndarray:
    sigma = fwhm_arcsec / (2.0 * math.sqrt(2.0 * math.log(2.0))) / pixscale
    r = np.arange(size) - size // 2
    rr = r[:, None] ** 2 + r[None, :] ** 2
    return np.exp(-rr / (2.0 * sigma * sigma)).astype(np.float32)


def moffat_psf(size: int, fwhm_arcsec: float, beta: float = 3.0, pixscale: float = PIXSCALE) -> np.ndarray:
    alpha = fwhm_arcsec / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0)) / pixscale
    r = np.arange(size) - size // 2
    rr = r[:, None] ** 2 + r[None, :] ** 2
    return ((1.0 + rr / (alpha * alpha)) ** (-beta)).astype(np.float32)


def pixel_radius(height: int, width: int, pixscale: float = PIXSCALE,
                 center_x: float = 0.0, center_y: float = 0.0) -> np.ndarray:
    """Distance of each pixel centre from the lens at the origin (row 0 = smallest y)."""
    x = center_x + (np.arange(width) - 0.5 * (width - 1)) * pixscale
    y = center_y + (np.arange(height) - 0.5 * (height - 1)) * pixscale
    return np.sqrt(x[None, :] ** 2 + y[:, None] ** 2)


def annulus_mask(height: int, width: int, rmin: float, rmax: float, pixscale: float = PIXSCALE) -> np.ndarray:
    r = pixel_radius(height, width, pixscale)
    return (r >= rmin) & (r <= rmax)


# ---------------------------------------------------------------------------
# Workload definitions.
# ---------------------------------------------------------------------------

@dataclass
class SystemSpec:
    name: str
    height: int
    width: int
    nsub: int
    psf: np.ndarray                 # float32, odd square
    truth: np.ndarray               # float32 [17]
    prior: Prior
    mask: np.ndarray                # bool [H, W]
    mock_seed: int
    noise_from_source_only: bool    # sigma from the lensed-source component only
    pixscale: float = PIXSCALE
    center_x: float = 0.0
    center_y: float = 0.0


@dataclass
class Observation:
    """A mock observation: float32 data and weights ready for either implementation."""
    spec: SystemSpec
    data: np.ndarray                # float32 [H, W]
    weight: np.ndarray              # float32 [H, W], 1/sigma^2 inside the mask, 0 outside
    sigma: float


# C0: 64x64 SIS with a circular n = 1 source; free theta_E, source position, R_e, I_e.
C0_FIXED = np.array([1.0, 1.0, 0.0, 0.0, 0.0,
                     0.0, 1.0, 1.0, 1.0, 0.0,
                     0.0, 0.0, 1.0, 0.2, 1.0, 1.0, 0.0])
C0_PRIORS = {0: (0.5, 1.5), 10: (-0.2, 0.2), 11: (-0.2, 0.2), 12: (0.5, 2.0), 13: (0.1, 0.3)}
C0_MOCK_SEED, C0_POINT_SEED = 1505, 1

# C1: 200x200 SIE + shear + Sersic lens light + elliptical Sersic source.
C1_TRUTH = np.array([1.2, 0.75, math.pi / 4, 0.05, 0.5,
                     0.1, 1.5, 4.0, 0.8, 0.9,
                     0.10, -0.05, 1.0, 0.2, 1.5, 0.7, 1.0])
C1_PRIORS = {0: (0.8, 1.5), 1: (0.5, 1.0), 2: (0.0, math.pi), 3: (0.0, 0.1), 4: (0.0, math.pi),
             5: (0.02, 0.2), 6: (0.5, 2.0), 7: (2.0, 6.0), 8: (0.6, 1.0), 9: (0.0, math.pi),
             10: (-0.5, 0.5), 11: (-0.5, 0.5), 12: (0.5, 2.0), 13: (0.05, 0.5), 14: (0.5, 4.0),
             15: (0.3, 1.0), 16: (0.0, math.pi)}
C1_MOCK_SEED, C1_POINT_SEED = 7674, 2
C2_BASE_SEED, C3_SEED, C4_SEED = 3, 4, 5


def c0_spec() -> SystemSpec:
    rng = np.random.default_rng(C0_MOCK_SEED)
    truth = C0_FIXED.copy()
    truth[10], truth[11] = rng.uniform(-0.2, 0.2, size=2)
    return SystemSpec("c0_64x64_sis_sub2_gauss7", 64, 64, 2, gaussian_psf(7, 0.1),
                      truth.astype(np.float32), _prior(C0_PRIORS, C0_FIXED),
                      np.ones((64, 64), bool), C0_MOCK_SEED, False)


def c1_spec() -> SystemSpec:
    return SystemSpec("c1_200x200_sie_shear_sersic_sub4_moffat21", 200, 200, 4, moffat_psf(21, 0.1, 3.0),
                      C1_TRUTH.astype(np.float32), _prior(C1_PRIORS, C1_TRUTH),
                      annulus_mask(200, 200, 0.3, 3.0), C1_MOCK_SEED, True)


C2_SIDES = (64, 100, 150, 200, 300)


def c2_specs(n_systems: int = 16) -> List[SystemSpec]:
    """16 systems of mixed size and subsampling, each with its own PSF width and truth."""
    out = []
    prior = _prior(C1_PRIORS, C1_TRUTH)
    for s in range(n_systems):
        rng = np.random.default_rng(C2_BASE_SEED + s)
        side = int(rng.choice(C2_SIDES))
        nsub = int(rng.integers(2, 9))
        fwhm = float(rng.uniform(0.08, 0.15))
        truth = prior.from_unit(rng.random(NPAR)).astype(np.float32)
        rmax = min(3.0, 0.4 * side * PIXSCALE)
        out.append(SystemSpec(f"c2_sys{s:02d}_{side}x{side}_sub{nsub}", side, side, nsub,
                              moffat_psf(21, fwhm, 3.0), truth, prior,
                              annulus_mask(side, side, 0.3, rmax), C2_BASE_SEED + 1000 + s, True))
    return out


def points(spec: SystemSpec, n: int, seed: int) -> np.ndarray:
    """n parameter points (float32 [n, 17]) drawn from the spec's prior."""
    return spec.prior.sample(n, seed)


def make_observation(spec: SystemSpec, render_noiseless: Callable[[np.ndarray], np.ndarray]) -> Observation:
    """Mock = noiseless model + Gaussian noise, stored in float32.

    ``render_noiseless(theta)`` must return the PSF-convolved model image [H, W]
    for a float32 parameter vector. sigma is 1 % of the peak of the full model
    image, or of the lensed source alone when ``noise_from_source_only`` (so that
    a cuspy lens-light centre does not set the noise level).
    """
    model = np.asarray(render_noiseless(spec.truth), dtype=np.float64)
    if spec.noise_from_source_only:
        t = spec.truth.copy()
        t[5] = 0.0
        peak = float(np.max(np.asarray(render_noiseless(t), dtype=np.float64)))
    else:
        peak = float(np.max(model))
    sigma = 0.01 * peak
    rng = np.random.default_rng(spec.mock_seed)
    eps = rng.standard_normal(model.shape)
    data = (model + sigma * eps).astype(np.float32)
    weight = np.where(spec.mask, 1.0 / (sigma * sigma), 0.0).astype(np.float32)
    return Observation(spec, data, weight, sigma)


# General model of Sec. 5 (a lens with a companion): two SIEs with free centres,
# an external shear, two host components, the companion's light, a lensed
# source and a flat sky: 41 parameters, layout of lensed_model (per SIE
# x, y, theta_E, q, phi; shear gamma, phi; per Sersic x, y, I_e, R_e, n, q, phi;
# sky). Planes: three foreground components, then the lensed source.
GENERAL_41_PLANES = ["foreground", "foreground", "foreground", "lensed"]


def general_model_points(n: int, seed: int) -> np.ndarray:
    """n parameter points (float32 [n, 41]) of the companion model, uniform in
    ranges around a main lens of theta_E ~ 1.1 arcsec and a companion 0.6-1.0
    arcsec away."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n):
        p = [rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05), rng.uniform(0.9, 1.3), rng.uniform(0.5, 1.0),
             rng.uniform(0, math.pi)]                                              # main SIE
        a = rng.uniform(0, 2 * math.pi)
        r = rng.uniform(0.6, 1.0)
        cx, cy = r * math.cos(a), r * math.sin(a)
        p += [cx, cy, rng.uniform(0.1, 0.4), rng.uniform(0.6, 1.0), rng.uniform(0, math.pi)]   # companion SIE
        p += [rng.uniform(0, 0.08), rng.uniform(0, math.pi)]                                  # shear
        p += [p[0], p[1], rng.uniform(0.05, 0.2), rng.uniform(0.5, 1.5), rng.uniform(2, 5), rng.uniform(0.6, 1),
              rng.uniform(0, math.pi)]                                                         # host, extended
        p += [p[0], p[1], rng.uniform(0.2, 0.6), rng.uniform(0.1, 0.3), rng.uniform(0.5, 1.5), rng.uniform(0.6, 1),
              rng.uniform(0, math.pi)]                                                         # host, compact
        p += [cx, cy, rng.uniform(0.05, 0.2), rng.uniform(0.1, 0.4), rng.uniform(1, 4), rng.uniform(0.6, 1),
              rng.uniform(0, math.pi)]                                                         # companion light
        p += [rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), rng.uniform(0.5, 2), rng.uniform(0.05, 0.4),
              rng.uniform(0.5, 4), rng.uniform(0.3, 1), rng.uniform(0, math.pi)]               # source
        p += [rng.uniform(0.0, 0.5)]                                                           # sky
        rows.append(p)
    return np.array(rows, np.float32)
