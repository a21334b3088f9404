"""GPU parity of general models (Sec. 5: several SIEs with free centres, an
external shear, several Sersic components in the image or source plane, a flat
sky) against the FP64 oracle: images with the midpoint and a Gauss-Kronrod
rule, batched log L over two systems, the base model against the 17-parameter
path, invalid points and invalid models."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1505_07674_amd as lensed
from paper_1505_07674_amd import mocks
from paper_1505_07674_amd.binding import LensedError

from helpers import f32, loglike_tolerance
from test_gpu_grad import small_spec

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
PLANES = {"foreground": "image", "lensed": "source"}


def say(msg):
    print(msg, flush=True)


def models(n_sie, planes, shear=True, sky=False):
    return (lensed.Model(n_sie, planes, shear=shear, sky=sky),
            oracle.Model(n_sie, [PLANES[p] for p in planes], shear=shear, sky=sky))


def osys(spec, data=None, weight=None, rule=None):
    return oracle.System(spec.height, spec.width, f32(spec.pixscale), spec.nsub, spec.psf.astype(np.float64), data,
                         weight, center_x=f32(spec.center_x), center_y=f32(spec.center_y), rule=rule)


def gsys(spec, data=None, weight=None, rule="sub"):
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)
    return lensed.System(t(spec.psf), t(data), t(weight), pixscale=spec.pixscale, nsub=spec.nsub,
                         height=spec.height, width=spec.width, center=(spec.center_x, spec.center_y), rule=rule)


def companion_points(n, seed, sky=True):
    """A lens with a companion (two SIEs), shear, two host components, the
    companion's light and a source, plus the sky: 41 parameters."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n):
        p = []
        p += [rng.uniform(-0.05, 0.05), rng.uniform(-0.05, 0.05), rng.uniform(0.9, 1.3), rng.uniform(0.5, 1.0),
              rng.uniform(0, math.pi)]                                   # main SIE
        cx, cy = rng.uniform(0.6, 1.0) * np.array([math.cos(a := rng.uniform(0, 6.28)), math.sin(a)])
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
        if sky:
            p += [rng.uniform(0.0, 0.5)]
        rows.append(p)
    return np.array(rows, np.float32)


PLANES_41 = ["foreground", "foreground", "foreground", "lensed"]


@pytest.mark.parametrize("rule", ["sub", "g3k7"])
def test_general_model_images_match_the_oracle(rule):
    spec = small_spec(H=48, W=44, N=3)
    gm, om = models(2, PLANES_41, sky=True)
    assert gm.n_params == om.n_params == 41
    g, o = gsys(spec, rule=rule), osys(spec, rule=None if rule == "sub" else rule)
    say(f"general model (2 SIEs, 4 Sersics, sky) images, rule {rule}")
    for t in companion_points(6, seed=70):
        for psf in (False, True):
            img = lensed.render_model(torch.from_numpy(t).to(DEV), g, gm, apply_psf=psf).cpu().numpy()
            ref = oracle.render_model(o, om, t.astype(np.float64), apply_psf=psf)
            err = np.max(np.abs(img.astype(np.float64) - ref)) / np.max(np.abs(ref))
            say(f"  rule {rule} psf {psf}: max error / peak {err:.2e}")
            # float64 rays; the Sersic profiles' fractional powers of two in float32
            assert err <= 1e-6, (rule, psf, err)


def test_general_model_loglike_matches_the_oracle():
    specs = [small_spec(), small_spec(H=36, W=44, N=2, center=(-0.04, 0.06))]
    gm, om = models(2, PLANES_41, sky=True)
    truth = companion_points(1, seed=71)[0]
    gs, os_ = [], []
    for s in specs:
        model = oracle.render_model(osys(s), om, truth.astype(np.float64))
        sigma = 0.01 * model.max()
        data = (model + sigma * np.random.default_rng(s.width).standard_normal(model.shape)).astype(np.float32)
        weight = np.full(model.shape, 1.0 / sigma ** 2, np.float32)
        gs.append(gsys(s, data, weight))
        os_.append(osys(s, data.astype(np.float64), weight.astype(np.float64)))
    pts = companion_points(24, seed=72)
    som = np.arange(24, dtype=np.int32) % 2
    say("general model log L, 24 points, 2 systems")
    ll = lensed.loglike_model_batch(torch.from_numpy(pts).to(DEV), som, gs, gm).cpu().numpy()
    ref = np.array([oracle.loglike_model(os_[som[i]], om, pts[i].astype(np.float64)) for i in range(24)])
    tol = np.array([loglike_tolerance(ref[i:i + 1], gs[som[i]].weight.cpu().numpy())[0] for i in range(24)])
    err = np.abs(ll - ref) / tol
    say(f"log L errors / bar: max {err.max():.3f}")
    assert np.all(err <= 1.0), (err, ref)


def test_the_base_model_matches_the_17_parameter_path():
    spec = small_spec()
    gm, om = models(1, ["foreground", "lensed"])
    pts = mocks.points(spec, 6, seed=73).astype(np.float32)
    g = gsys(spec)
    for t in pts:
        p = np.concatenate([[0.0, 0.0], t[0:3], t[3:5], [0.0, 0.0], t[5:10], t[10:17]]).astype(np.float32)
        a = lensed.render_model(torch.from_numpy(p).to(DEV), g, gm).cpu().numpy().astype(np.float64)
        b = lensed.render(torch.from_numpy(t).to(DEV), g).cpu().numpy().astype(np.float64)
        ref = oracle.render(osys(spec), t.astype(np.float64))
        assert np.max(np.abs(a - ref)) <= 1e-6 * np.max(np.abs(ref))
        assert np.max(np.abs(b - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_invalid_points_and_models():
    spec = small_spec()
    gm, _ = models(2, PLANES_41, sky=True)
    g = gsys(spec, np.zeros((40, 36), np.float32), np.ones((40, 36), np.float32))
    pts = companion_points(3, seed=74)
    pts[1, 3] = 1.5                          # q of the main SIE outside (0, 1]
    ll = lensed.loglike_model_batch(torch.from_numpy(pts).to(DEV), np.zeros(3, np.int32), [g], gm).cpu().numpy()
    assert np.isfinite(ll[0]) and np.isnan(ll[1]) and np.isfinite(ll[2])
    with pytest.raises(ValueError):
        lensed.Model(9, ["lensed"])
    with pytest.raises(ValueError):
        lensed.render_model(torch.zeros(17, device=DEV), g, gm)
