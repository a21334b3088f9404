"""GPU parity of the magnitude parametrisation (Sec. 4.1: a Sersic component's
amplitude is set by its total magnitude) against the FP64 oracle: model images,
log L, the adjoint gradient with respect to the magnitudes (and the extra
d I_e / d R_e, d I_e / d n terms), a batch that mixes systems in both modes, and
the argument checks."""
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


def osys(spec, obs=None, amplitude="magnitude"):
    return oracle.System(spec.height, spec.width, f32(spec.pixscale), spec.nsub, spec.psf.astype(np.float64),
                         None if obs is None else obs.data.astype(np.float64),
                         None if obs is None else obs.weight.astype(np.float64),
                         center_x=f32(spec.center_x), center_y=f32(spec.center_y), amplitude=amplitude,
                         zero_point=ZP)


def gsys(spec, obs=None, amplitude="magnitude"):
    t = lambda a: None if a is None else torch.from_numpy(a).to(DEV)
    return lensed.System(t(spec.psf), t(None if obs is None else obs.data), t(None if obs is None else obs.weight),
                         pixscale=spec.pixscale, nsub=spec.nsub, height=spec.height, width=spec.width,
                         center=(spec.center_x, spec.center_y), amplitude=amplitude, zero_point=ZP)


def magnitude_points(spec, n, seed):
    pts = mocks.points(spec, n, seed=seed).astype(np.float32)
    rng = np.random.default_rng(seed + 1000)
    pts[:, 5] = rng.uniform(16.5, 19.0, n)
    pts[:, 12] = rng.uniform(20.0, 23.0, n)
    return pts


def magnitude_truth(spec):
    t = spec.truth.astype(np.float64).copy()
    for k in (5, 12):      # the same fluxes as the intensity truth
        unit = oracle.intensity_from_magnitude(ZP, t[k + 1], t[k + 2], ZP)
        t[k] = ZP - 2.5 * math.log10(t[k] / unit)
    return t.astype(np.float32)


def test_magnitude_images_match_the_oracle():
    spec = small_spec(H=48, W=44, N=3)
    pts = magnitude_points(spec, 12, seed=41)
    pts[0] = magnitude_truth(spec)
    os_, gs = osys(spec), gsys(spec)
    say("magnitude render, 48x44 sub3, 12 points")
    for t in pts:
        img = lensed.render(torch.from_numpy(t).to(DEV), gs).cpu().numpy().astype(np.float64)
        ref = oracle.render(os_, t.astype(np.float64))
        assert np.max(np.abs(img - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_magnitude_truth_renders_the_intensity_truth():
    spec = small_spec()
    a = lensed.render(torch.from_numpy(magnitude_truth(spec)).to(DEV), gsys(spec)).cpu().numpy()
    b = lensed.render(torch.from_numpy(spec.truth).to(DEV), gsys(spec, amplitude="intensity")).cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(b))


def test_magnitude_loglike_and_gradient_match_the_oracle():
    spec = small_spec()
    truth = magnitude_truth(spec)
    ref_sys = osys(spec)
    obs = mocks.make_observation(spec, lambda t: oracle.render(ref_sys, np.asarray(truth, np.float64)))
    pts = magnitude_points(spec, 16, seed=43)
    rng = np.random.default_rng(44)
    # around the truth, far enough out that log L is well above the float32 noise
    # floor of a 1440-pixel image (the truth itself is covered by the render test)
    near = np.repeat(truth[None], 8, axis=0)
    near[:, [5, 12]] += rng.choice([-1.0, 1.0], (8, 2)) * rng.uniform(0.4, 0.8, (8, 2))
    near[:, [6, 7, 13, 14]] *= (1 + rng.choice([-1.0, 1.0], (8, 4)) * rng.uniform(0.1, 0.2, (8, 4)))
    pts = np.concatenate([pts, near.astype(np.float32)]).astype(np.float32)
    g = gsys(spec, obs)
    tp = torch.from_numpy(pts).to(DEV)
    say("magnitude log L and gradient, 24 points")
    ll, gr = lensed.loglike_grad(tp, g)
    ll, gr = ll.cpu().numpy(), gr.cpu().numpy().astype(np.float64)
    lb = lensed.loglike_batch(tp, np.zeros(len(pts), np.int32), [g]).cpu().numpy()
    assert np.allclose(ll, lb, rtol=1e-12, atol=0)
    rll, rg = oracle_grads(osys(spec, obs), pts)
    err = np.abs(ll - rll) / loglike_tolerance(rll, obs.weight)
    say(f"log L errors / bar: max {err.max():.3f}; log L near the truth {rll[16:].max():.1f} .. {rll[16:].min():.1f}")
    assert np.all(err <= 1.0), (err, rll)
    rel = np.linalg.norm(gr - rg, axis=1) / np.linalg.norm(rg, axis=1)
    assert rel.max() <= 1e-4, (rel.max(), int(np.argmax(rel)))


def test_one_batch_mixes_intensity_and_magnitude_systems():
    spec = small_spec()
    obs = mocks.make_observation(spec, lambda t: oracle.render(osys(spec, amplitude="intensity"),
                                                               np.asarray(t, np.float64)))
    g_int, g_mag = gsys(spec, obs, amplitude="intensity"), gsys(spec, obs)
    pi = mocks.points(spec, 20, seed=45).astype(np.float32)
    pm = magnitude_points(spec, 20, seed=46)
    th = torch.from_numpy(np.concatenate([pi, pm])).to(DEV)
    sop = np.array([0] * 20 + [1] * 20, np.int32)
    both = lensed.loglike_batch(th, sop, [g_int, g_mag]).cpu().numpy()
    a = lensed.loglike_batch(th[:20], np.zeros(20, np.int32), [g_int]).cpu().numpy()
    b = lensed.loglike_batch(th[20:], np.zeros(20, np.int32), [g_mag]).cpu().numpy()
    assert np.allclose(both, np.concatenate([a, b]), rtol=1e-12, atol=0)
    ref = [oracle.loglike(osys(spec, obs, "intensity"), t.astype(np.float64)) for t in pi[:4]]
    ref += [oracle.loglike(osys(spec, obs), t.astype(np.float64)) for t in pm[:4]]
    got = np.concatenate([both[:4], both[20:24]])
    assert np.all(np.abs(got - np.array(ref)) <= loglike_tolerance(np.array(ref), obs.weight))


def test_amplitude_arguments_are_checked():
    spec = small_spec()
    g = gsys(spec)
    t = torch.from_numpy(magnitude_points(spec, 1, seed=47)[0]).to(DEV)
    g.c_struct.amplitude = 2
    with pytest.raises(LensedError):
        lensed.render(t, g)
    g.c_struct.amplitude = 1
    g.c_struct.zero_point = float("nan")
    with pytest.raises(LensedError):
        lensed.render(t, g)
    with pytest.raises(ValueError):
        gsys(spec, amplitude="flux")
