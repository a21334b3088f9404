"""Gauss-Kronrod pixel integration (Sec. 3.1 Eq. 14; Sec. 4.5: g3k7, g5k11,
g7k15) on the GPU against the FP64 oracle with the same rule, through the C
ABI: model images before and after the PSF (the bars of the midpoint parity
tests), log L in the batched and the plain form, the adjoint gradient, and the
per-pixel error estimate |Kronrod - embedded Gauss|."""
import numpy as np
import pytest
import torch

import oracle
import paper_1505_07674_amd as lensed
from paper_1505_07674_amd import mocks

from helpers import loglike_tolerance, oracle_loglikes
from test_gpu_grad import oracle_grads

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
RULES = ["g3k7", "g5k11", "g7k15"]


def say(msg):
    print(msg, flush=True)


def spec_for(H=40, W=36, psf=None, pixscale=0.07, center=(0.1, -0.05)):
    base = mocks.c1_spec()
    psf = mocks.moffat_psf(7, 0.15, 3.0, pixscale) if psf is None else psf
    return mocks.SystemSpec(f"gk_{H}x{W}", H, W, 1, psf.astype(np.float32), base.truth, base.prior,
                            np.ones((H, W), bool), 77, False, pixscale=pixscale, center_x=center[0],
                            center_y=center[1])


def gsys(spec, rule, data=None, weight=None):
    return lensed.System(torch.from_numpy(spec.psf).to(DEV),
                         None if data is None else torch.from_numpy(data).to(DEV),
                         None if weight is None else torch.from_numpy(weight).to(DEV),
                         pixscale=spec.pixscale, height=spec.height, width=spec.width,
                         center=(spec.center_x, spec.center_y), rule=rule)


def osys(spec, rule, data=None, weight=None):
    return oracle.System(spec.height, spec.width, float(np.float32(spec.pixscale)), 1,
                         spec.psf.astype(np.float64), data, weight, center_x=float(np.float32(spec.center_x)),
                         center_y=float(np.float32(spec.center_y)), rule=rule)


def points(spec, n, seed):
    pts = mocks.points(spec, n, seed=seed)
    pts[0] = spec.truth
    pts[-1, 14] = 4.0          # a cuspy source...
    pts[-1, 13] = 0.06         # ...compact enough to trigger the float64 re-tracing
    return pts


@pytest.mark.parametrize("rule", RULES)
def test_gauss_kronrod_images_match_the_oracle(rule):
    say(f"{rule}: images")
    spec = spec_for()
    g, o = gsys(spec, rule), osys(spec, rule)
    for t in points(spec, 4, seed=61):
        for psf in (False, True):
            img = lensed.render(torch.from_numpy(t).to(DEV), g, apply_psf=psf).cpu().numpy().astype(np.float64)
            ref = oracle.render(o, t.astype(np.float64), apply_psf=psf)
            err = np.max(np.abs(img - ref)) / np.max(np.abs(ref))
            say(f"  apply_psf={psf}: pixel error {err:.3e} x peak")
            assert err <= 1e-5, (rule, psf, err, t.tolist())


@pytest.mark.parametrize("rule", RULES)
def test_gauss_kronrod_loglike_batched_and_plain(rule):
    say(f"{rule}: log L")
    spec = spec_for(H=32, W=30)
    o = osys(spec, rule)
    model = oracle.render(o, spec.truth.astype(np.float64))
    rng = np.random.default_rng(7)
    sigma = 0.01 * model.max()
    data = (model + sigma * rng.standard_normal(model.shape)).astype(np.float32)
    weight = np.full(model.shape, 1.0 / sigma ** 2, np.float32)
    g = gsys(spec, rule, data, weight)
    pts = points(spec, 6, seed=62)
    tp = torch.from_numpy(pts).to(DEV)
    ll = lensed.loglike_batch(tp, np.zeros(len(pts), np.int32), [g]).cpu().numpy()
    ref = oracle_loglikes(osys(spec, rule, data.astype(np.float64), weight.astype(np.float64)), pts)
    tol = loglike_tolerance(ref, weight)
    far = np.arange(1, len(pts))          # the truth row sits on the float32 noise floor of a small image
    assert np.all(np.abs(ll[far] - ref[far]) <= tol[far]), (ll - ref, tol)
    plain = np.array([lensed.loglike(tp[i], g).cpu().numpy()[0] for i in range(len(pts))])
    assert np.allclose(plain, ll, rtol=1e-5, atol=0)


@pytest.mark.parametrize("rule", RULES)
def test_gauss_kronrod_error_estimate(rule):
    say(f"{rule}: error estimate")
    spec = spec_for(H=24, W=26)
    g, o = gsys(spec, rule), osys(spec, rule)
    for t in points(spec, 3, seed=63):
        est = lensed.render_error(torch.from_numpy(t).to(DEV), g).cpu().numpy().astype(np.float64)
        ref = oracle.render_error(o, t.astype(np.float64))
        peak = np.max(np.abs(oracle.render(o, t.astype(np.float64), apply_psf=False)))
        assert np.all(est >= 0)
        # ||K - G| - |K_o - G_o|| <= |K - K_o| + |G - G_o|: two rule sums, each held to 1e-5 x peak
        err = np.max(np.abs(est - ref)) / peak
        say(f"  error map: {err:.3e} x peak")
        assert err <= 2e-5, (rule, err)


@pytest.mark.parametrize("rule", RULES)
def test_gauss_kronrod_gradient_matches_the_oracle(rule):
    """The adjoint with the rule's nodes and weights (and the weighted float64
    cusp re-tracing) against the oracle's dual-number gradient of the same rule."""
    say(f"{rule}: gradient")
    spec = spec_for(H=30, W=28)
    o = osys(spec, rule)
    model = oracle.render(o, spec.truth.astype(np.float64))
    rng = np.random.default_rng(8)
    sigma = 0.01 * model.max()
    data = (model + sigma * rng.standard_normal(model.shape)).astype(np.float32)
    weight = np.full(model.shape, 1.0 / sigma ** 2, np.float32)
    g = gsys(spec, rule, data, weight)
    pts = points(spec, 8, seed=64)[1:]             # away from the truth (noise-driven gradient there)
    tp = torch.from_numpy(np.ascontiguousarray(pts)).to(DEV)
    ll, gr = lensed.loglike_grad(tp, g)
    ll, gr = ll.cpu().numpy(), gr.cpu().numpy().astype(np.float64)
    lb = lensed.loglike_batch(tp, np.zeros(len(pts), np.int32), [g]).cpu().numpy()
    assert np.allclose(ll, lb, rtol=1e-12, atol=0)
    rll, rg = oracle_grads(osys(spec, rule, data.astype(np.float64), weight.astype(np.float64)), pts)
    rel = np.linalg.norm(gr - rg, axis=1) / np.linalg.norm(rg, axis=1)
    assert rel.max() <= 1e-4, (rule, rel)


def test_rules_are_validated():
    spec = spec_for(H=8, W=8)
    with pytest.raises(lensed.LensedError) as e:
        lensed.render_error(torch.from_numpy(spec.truth).to(DEV), gsys(spec, "sub"))
    assert e.value.status == 1
    with pytest.raises(ValueError):
        gsys(spec, "g9k19")
