"""GPU parity of composite models (Sec. 5: extra Sersic components and a flat
sky on top of the base model) against the FP64 oracle: images, batched log L of
models with 2 and 3 components and a sky over two systems, the one-component
case against the plain batch, and the argument checks."""
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


def say(msg):
    print(msg, flush=True)


def osys(spec, data=None, weight=None):
    return oracle.System(spec.height, spec.width, f32(spec.pixscale), spec.nsub, spec.psf.astype(np.float64), data,
                         weight, center_x=f32(spec.center_x), center_y=f32(spec.center_y))


def gsys(spec, data=None, weight=None):
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)
    return lensed.System(t(spec.psf), t(data), t(weight), pixscale=spec.pixscale, nsub=spec.nsub,
                         height=spec.height, width=spec.width, center=(spec.center_x, spec.center_y))


def components(spec, K, seed):
    """K points sharing the lens parameters of the first: extra light components."""
    pts = mocks.points(spec, K, seed=seed).astype(np.float32)
    pts[1:, :5] = pts[0, :5]
    return pts


def test_composite_images_match_the_oracle():
    spec = small_spec(H=44, W=40, N=3)
    o, g = osys(spec), gsys(spec)
    say("composite images, K = 1..3")
    for K, sky in ((1, 0.0), (2, 0.0), (3, 0.4)):
        th = components(spec, K, seed=90 + K)
        for psf in (False, True):
            img = lensed.render_composite(torch.from_numpy(th).to(DEV), g, sky=sky, apply_psf=psf)
            ref = oracle.render_composite(o, th.astype(np.float64), sky=float(np.float32(sky)), apply_psf=psf)
            err = np.max(np.abs(img.cpu().numpy().astype(np.float64) - ref)) / np.max(np.abs(ref))
            say(f"  K={K} apply_psf={psf}: pixel error {err:.3e} x peak")
            assert err <= 1e-5, (K, psf, err)


@pytest.mark.parametrize("K", [2, 3])
def test_composite_loglike_matches_the_oracle(K):
    specs = [small_spec(), small_spec(H=36, W=44, N=2, center=(-0.04, 0.06))]
    truth = components(specs[0], K, seed=100 + K)
    systems, osystems = [], []
    for s in specs:
        model = oracle.render_composite(osys(s), truth.astype(np.float64), sky=0.3)
        sigma = 0.01 * model.max()
        rng = np.random.default_rng(s.height)
        data = (model + sigma * rng.standard_normal(model.shape)).astype(np.float32)
        weight = np.full(model.shape, 1.0 / sigma ** 2, np.float32)
        systems.append(gsys(s, data, weight))
        osystems.append(osys(s, data.astype(np.float64), weight.astype(np.float64)))
    M = 12
    th = np.concatenate([components(specs[0], K, seed=200 + m) for m in range(M)]).astype(np.float32)
    sky = np.random.default_rng(5).uniform(0.0, 0.6, M).astype(np.float32)
    som = np.arange(M, dtype=np.int32) % 2
    say(f"composite log L, {M} models of {K} components, 2 systems")
    ll = lensed.loglike_composite(torch.from_numpy(th).to(DEV), K, som, systems,
                                  sky=torch.from_numpy(sky).to(DEV)).cpu().numpy()
    ref = np.array([oracle.loglike_composite(osystems[som[m]], th[m * K:(m + 1) * K].astype(np.float64),
                                             sky=float(sky[m])) for m in range(M)])
    tol = np.array([loglike_tolerance(ref[m:m + 1], systems[som[m]].weight.cpu().numpy())[0] for m in range(M)])
    err = np.abs(ll - ref) / tol
    say(f"log L errors / bar: max {err.max():.3f}")
    assert np.all(err <= 1.0), (err, ref)
    # the same call again replays the cached plan and gives the same numbers
    again = lensed.loglike_composite(torch.from_numpy(th).to(DEV), K, som, systems,
                                     sky=torch.from_numpy(sky).to(DEV)).cpu().numpy()
    assert np.array_equal(ll, again)


def test_one_component_without_sky_is_the_plain_batch():
    spec = small_spec()
    model = oracle.render(osys(spec), spec.truth.astype(np.float64))
    sigma = 0.01 * model.max()
    data = (model + sigma * np.random.default_rng(1).standard_normal(model.shape)).astype(np.float32)
    g = gsys(spec, data, np.full(model.shape, 1.0 / sigma ** 2, np.float32))
    pts = torch.from_numpy(mocks.points(spec, 30, seed=300).astype(np.float32)).to(DEV)
    a = lensed.loglike_composite(pts, 1, np.zeros(30, np.int32), [g]).cpu().numpy()
    b = lensed.loglike_batch(pts, np.zeros(30, np.int32), [g]).cpu().numpy()
    assert np.array_equal(a, b)


def test_composite_arguments_are_checked():
    spec = small_spec()
    g = gsys(spec, np.zeros((40, 36), np.float32), np.ones((40, 36), np.float32))
    th = torch.from_numpy(components(spec, 2, seed=400)).to(DEV)
    with pytest.raises(ValueError):
        lensed.loglike_composite(th, 3, [0], [g])
    with pytest.raises(LensedError):
        lensed.loglike_composite(th, 2, [1], [g])
    with pytest.raises(LensedError):
        lensed.render_composite(th, g, sky=float("nan"))


def test_multiband_log_likelihoods_add_over_bands():
    """Two bands (different grids, PSFs and noise) of composite models with
    their own amplitudes and skies: the GPU sum of the bands' log L against the
    oracle's, and against two single-band composite calls."""
    bands = [small_spec(), small_spec(H=36, W=44, N=3, psf=mocks.moffat_psf(9, 0.2, 3.0, 0.08), center=(-0.04, 0.06))]
    K, M = 2, 8
    truth = components(bands[0], K, seed=500)
    gs, os_ = [], []
    for i, s in enumerate(bands):
        model = oracle.render_composite(osys(s), truth.astype(np.float64), sky=0.1 * (i + 1))
        sigma = 0.01 * model.max()
        data = (model + sigma * np.random.default_rng(10 + i).standard_normal(model.shape)).astype(np.float32)
        weight = np.full(model.shape, 1.0 / sigma ** 2, np.float32)
        gs.append(gsys(s, data, weight))
        os_.append(osys(s, data.astype(np.float64), weight.astype(np.float64)))
    rows, skies = [], []
    rng = np.random.default_rng(11)
    for m in range(M):
        base = components(bands[0], K, seed=600 + m)
        for b in range(2):
            band = base.copy()
            band[:, [5, 12]] *= rng.uniform(0.7, 1.3, (K, 2)).astype(np.float32)   # colours differ per band
            rows.append(band)
            skies.append(rng.uniform(0.0, 0.3))
    th = np.concatenate(rows).astype(np.float32)
    sky = np.array(skies, np.float32)
    say(f"multi-band log L: {M} models, 2 bands, {K} components")
    ll = lensed.loglike_multiband(torch.from_numpy(th).to(DEV), gs, K, sky=torch.from_numpy(sky).to(DEV)).cpu().numpy()
    ref = np.array([oracle.loglike_multiband(os_, [th[(2 * m + b) * K:(2 * m + b + 1) * K].astype(np.float64)
                                                   for b in range(2)], [float(sky[2 * m + b]) for b in range(2)])
                    for m in range(M)])
    nw = sum(int(np.count_nonzero(g.weight.cpu().numpy())) for g in gs)
    tol = 1e-6 * np.maximum(np.abs(ref), nw / 2.0)
    assert np.all(np.abs(ll - ref) <= tol), (ll - ref, tol)
    per_band = []
    for b in range(2):
        idx = np.concatenate([np.arange((2 * m + b) * K, (2 * m + b + 1) * K) for m in range(M)])
        per_band.append(lensed.loglike_composite(torch.from_numpy(th[idx]).to(DEV), K, np.zeros(M, np.int32), [gs[b]],
                                                 sky=torch.from_numpy(sky[b::2].copy()).to(DEV)).cpu().numpy())
    assert np.allclose(ll, per_band[0] + per_band[1], rtol=1e-12, atol=0)


def _composite_case(K, n_models, seed):
    spec = small_spec(H=40, W=36, N=2)
    truth = components(spec, K, seed=seed)
    sky_true = 0.3
    o = osys(spec)
    model = oracle.render_composite(o, truth.astype(np.float64), sky=float(np.float32(sky_true)))
    sigma = 0.01 * model.max()
    rng = np.random.default_rng(seed)
    data = (model + sigma * rng.standard_normal(model.shape)).astype(np.float32)
    weight = ((rng.random(model.shape) < 0.85) / sigma ** 2).astype(np.float32)
    pts = np.concatenate([components(spec, K, seed=seed + 1 + m) for m in range(n_models)])
    skies = (sky_true + 0.2 * rng.standard_normal(n_models)).astype(np.float32)
    return spec, data, weight, pts, skies


def test_composite_gradient_with_one_component_is_the_17_parameter_gradient():
    spec, data, weight, pts, _ = _composite_case(1, 6, seed=310)
    g = gsys(spec, data, weight)
    tp = torch.from_numpy(pts).to(DEV)
    say("composite gradient, one component, no sky, against lensed_loglike_grad")
    ll, gr, gs = lensed.loglike_composite_grad(tp, 1, g)
    ll1, gr1 = lensed.loglike_grad(tp, g)
    assert gs is None
    assert np.array_equal(ll.cpu().numpy(), ll1.cpu().numpy())
    assert np.array_equal(gr.cpu().numpy(), gr1.cpu().numpy())


@pytest.mark.parametrize("K", [2, 3])
def test_composite_gradient_matches_the_oracle(K):
    """Component k's gradient is the 17-parameter gradient of the oracle on the
    data minus the other components and the sky (the residual is the same); the
    sky's is a Richardson difference of the oracle's composite log L."""
    n_models = 3
    spec, data, weight, pts, skies = _composite_case(K, n_models, seed=320 + K)
    g = gsys(spec, data, weight)
    tp = torch.from_numpy(pts).to(DEV)
    say(f"composite gradient, K = {K}, {n_models} models with a sky")
    ll, gr, gs = lensed.loglike_composite_grad(tp, K, g, sky=torch.from_numpy(skies).to(DEV))
    ll, gr, gs = ll.cpu().numpy(), gr.cpu().numpy().astype(np.float64), gs.cpu().numpy().astype(np.float64)
    o = osys(spec, data.astype(np.float64), weight.astype(np.float64))
    px2 = float(o.pixscale) ** 2
    for m in range(n_models):
        th = pts[m * K:(m + 1) * K].astype(np.float64)
        sky = float(skies[m])
        ref_ll = oracle.loglike_composite(o, th, sky=sky)
        assert abs(ll[m] - ref_ll) <= loglike_tolerance(np.array([ref_ll]), weight)[0], (m, ll[m], ref_ll)
        for k in range(K):
            others = sum(oracle.render(o, th[j]) for j in range(K) if j != k) + sky * px2
            ok = osys(spec, (data.astype(np.float64) - others).reshape(-1), weight.astype(np.float64))
            _, ref_g = oracle.loglike_grad(ok, th[k])
            got = gr[m * K + k]
            rel = np.linalg.norm(got - ref_g) / np.linalg.norm(ref_g)
            say(f"  model {m} component {k}: relative gradient error {rel:.2e}")
            assert rel <= 1e-4, (m, k, rel)
        h = 1e-3 * max(abs(sky), 1.0)
        f = lambda s: oracle.loglike_composite(o, th, sky=s)
        d1 = (f(sky + h) - f(sky - h)) / (2 * h)
        d2 = (f(sky + h / 2) - f(sky - h / 2)) / h
        ref_sky = (4 * d2 - d1) / 3
        # bar: 1e-4 of the sum of the terms' magnitudes, px^2 sum |w (d - L*)|
        resid = data.astype(np.float64) - oracle.render_composite(o, th, sky=sky)
        scale = px2 * np.sum(np.abs(weight.astype(np.float64) * resid))
        say(f"  model {m} sky: {gs[m]:.6g} vs {ref_sky:.6g} (scale {scale:.3g})")
        assert abs(gs[m] - ref_sky) <= 1e-4 * scale, (m, gs[m], ref_sky, scale)


def test_composite_gradient_arguments():
    spec, data, weight, pts, skies = _composite_case(2, 2, seed=330)
    g = gsys(spec, data, weight)
    tp = torch.from_numpy(pts).to(DEV)
    with pytest.raises(ValueError):
        lensed.loglike_composite_grad(tp[:3], 2, g)
    from paper_1505_07674_amd.binding import lib
    import ctypes
    rc = lib().lensed_loglike_composite_grad(lensed.default_context(0).handle, ctypes.byref(g.c_struct),
                                             ctypes.c_void_p(tp.data_ptr()), 2,
                                             ctypes.c_void_p(torch.from_numpy(skies).to(DEV).data_ptr()), 2,
                                             ctypes.c_void_p(torch.empty(2, dtype=torch.float64, device=DEV).data_ptr()),
                                             ctypes.c_void_p(torch.empty(4 * 17, device=DEV).data_ptr()), None, None)
    assert rc == 1   # LENSED_INVALID_ARGUMENT: a sky without grad_sky
