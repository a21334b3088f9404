"""GPU parity of image-plane source positions (Sec. 5: an image-plane point is
mapped to the source plane by the lens equation and becomes the source centre)
against the FP64 oracle: model images, log L, the adjoint gradient with respect
to the image-plane point (and the extra d beta / d lens-parameter terms), the
combination with magnitudes, and the argument check."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1505_07674_amd as lensed
from paper_1505_07674_amd import mocks
from paper_1505_07674_amd.binding import LensedError

from helpers import f32, loglike_tolerance
from test_gpu_grad import oracle_grads, small_spec

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
ZP = 25.0


def say(msg):
    print(msg, flush=True)


def osys(spec, obs=None, amplitude="intensity"):
    return oracle.System(spec.height, spec.width, f32(spec.pixscale), spec.nsub, spec.psf.astype(np.float64),
                         None if obs is None else obs.data.astype(np.float64),
                         None if obs is None else obs.weight.astype(np.float64),
                         center_x=f32(spec.center_x), center_y=f32(spec.center_y), amplitude=amplitude,
                         zero_point=ZP, source_position="image")


def gsys(spec, obs=None, amplitude="intensity"):
    t = lambda a: None if a is None else torch.from_numpy(a).to(DEV)
    return lensed.System(t(spec.psf), t(None if obs is None else obs.data), t(None if obs is None else obs.weight),
                         pixscale=spec.pixscale, nsub=spec.nsub, height=spec.height, width=spec.width,
                         center=(spec.center_x, spec.center_y), amplitude=amplitude, zero_point=ZP,
                         source_position="image")


def image_points(spec, n, seed):
    """Prior points whose slots 10, 11 are image-plane positions near the
    Einstein ring (where the images of a source are)."""
    pts = mocks.points(spec, n, seed=seed).astype(np.float32)
    rng = np.random.default_rng(seed + 500)
    r = pts[:, 0] * rng.uniform(0.8, 1.2, n)
    a = rng.uniform(0.0, 2.0 * math.pi, n)
    pts[:, 10] = r * np.cos(a)
    pts[:, 11] = r * np.sin(a)
    return pts


def test_image_plane_images_match_the_oracle():
    spec = small_spec(H=48, W=44, N=3)
    o, g = osys(spec), gsys(spec)
    say("image-plane source positions: render, 12 points")
    for t in image_points(spec, 12, seed=81):
        img = lensed.render(torch.from_numpy(t).to(DEV), g).cpu().numpy().astype(np.float64)
        ref = oracle.render(o, t.astype(np.float64))
        assert np.max(np.abs(img - ref)) <= 1e-5 * np.max(np.abs(ref)), t.tolist()


@pytest.mark.parametrize("amplitude", ["intensity", "magnitude"])
def test_image_plane_loglike_and_gradient_match_the_oracle(amplitude):
    spec = small_spec()
    truth = image_points(spec, 1, seed=82)[0]
    if amplitude == "magnitude":
        truth[5], truth[12] = 18.0, 21.0
    ref_sys = osys(spec, amplitude=amplitude)
    obs = mocks.make_observation(spec, lambda t: oracle.render(ref_sys, np.asarray(truth, np.float64)))
    pts = image_points(spec, 20, seed=83)
    if amplitude == "magnitude":
        rng = np.random.default_rng(84)
        pts[:, 5] = rng.uniform(16.5, 19.0, len(pts))
        pts[:, 12] = rng.uniform(20.0, 23.0, len(pts))
    g = gsys(spec, obs, amplitude)
    tp = torch.from_numpy(pts).to(DEV)
    say(f"image-plane source positions ({amplitude}): log L and gradient, 20 points")
    ll, gr = lensed.loglike_grad(tp, g)
    ll, gr = ll.cpu().numpy(), gr.cpu().numpy().astype(np.float64)
    lb = lensed.loglike_batch(tp, np.zeros(len(pts), np.int32), [g]).cpu().numpy()
    assert np.allclose(ll, lb, rtol=1e-12, atol=0)
    rll, rg = oracle_grads(osys(spec, obs, amplitude), pts)
    err = np.abs(ll - rll) / loglike_tolerance(rll, obs.weight)
    say(f"log L errors / bar: max {err.max():.3f} at point {int(np.argmax(err))}")
    assert np.all(err <= 1.0), (err, rll)
    rel = np.linalg.norm(gr - rg, axis=1) / np.linalg.norm(rg, axis=1)
    assert rel.max() <= 1e-4, (rel.max(), int(np.argmax(rel)))


def test_source_position_argument_is_checked():
    spec = small_spec()
    g = gsys(spec)
    t = torch.from_numpy(image_points(spec, 1, seed=85)[0]).to(DEV)
    g.c_struct.source_position = 2
    with pytest.raises(LensedError):
        lensed.render(t, g)
    with pytest.raises(ValueError):
        lensed.System(torch.from_numpy(spec.psf).to(DEV), pixscale=0.05, height=8, width=8, source_position="sky")
