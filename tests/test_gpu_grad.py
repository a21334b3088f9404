"""GPU adjoint (lensed_loglike_grad) against the FP64 oracle's exact gradient
(forward-mode dual numbers) and against central finite differences of the
oracle's log L.

Bar (per point): ||g_gpu - g_ref||_2 <= 1e-4 ||g_ref||_2, and the returned
log L within the log-likelihood bar of the forward parity tests. At the truth of
a mock (the likelihood maximum) g_ref is only the noise-driven gradient, of the
order of the Fisher scale sqrt(sum_i w_i (dL*_i/dtheta)^2); there the float32
model error (|dL*|/sigma ~ 3e-5 per pixel, partly correlated with dL*/dtheta)
sets a floor near 1e-4 to 1e-3 of ||g_ref||, and the bar is 1e-3.
"""
import numpy as np
import pytest
import torch
from concurrent.futures import ThreadPoolExecutor

import oracle
import paper_1505_07674_amd as lensed
from paper_1505_07674_amd import mocks

from helpers import golden, golden_file, loglike_tolerance, observation, oracle_system

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def gpu_system(spec, obs):
    return lensed.System(torch.from_numpy(spec.psf).to(DEV), torch.from_numpy(obs.data).to(DEV),
                         torch.from_numpy(obs.weight).to(DEV), pixscale=spec.pixscale, nsub=spec.nsub,
                         center=(spec.center_x, spec.center_y))


def oracle_grads(osys, pts):
    with ThreadPoolExecutor(max_workers=8) as ex:
        res = list(ex.map(lambda t: oracle.loglike_grad(osys, np.asarray(t, np.float64)), pts))
    return np.array([r[0] for r in res]), np.array([r[1] for r in res])


def check(spec, obs, pts, tol=1e-4, truth_rows=(), loglike_bar=True):
    """Gradient bar at every point (1e-3 at the truth rows, where the gradient is
    noise-driven; see the module docstring); the log L bar against the oracle
    away from the truth rows (on a ~1e3-pixel image the float32 model noise at
    the truth, about 2 sqrt(N_w) |dL*/sigma|, reaches the N_w/2 x 1e-6 floor;
    loglike_bar=False skips it for images of a few tens of pixels, where one
    pixel's float32 error, within the image bar, is not averaged), and
    everywhere the log L of the gradient plan equals the batched log L of the
    same points."""
    gsys = gpu_system(spec, obs)
    tp = torch.from_numpy(np.ascontiguousarray(pts)).to(DEV)
    ll, g = lensed.loglike_grad(tp, gsys)
    lb = lensed.loglike_batch(tp, np.zeros(len(pts), np.int32), [gsys]).cpu().numpy()
    ll, g = ll.cpu().numpy(), g.cpu().numpy().astype(np.float64)
    assert np.allclose(ll, lb, rtol=1e-12, atol=0)
    rll, rg = oracle_grads(oracle_system(spec, obs), pts)
    far = np.setdiff1d(np.arange(len(pts)), truth_rows)
    if loglike_bar:
        assert np.all(np.abs(ll[far] - rll[far]) <= loglike_tolerance(rll[far], obs.weight))
    rel = np.linalg.norm(g - rg, axis=1) / np.linalg.norm(rg, axis=1)
    bar = np.full(len(pts), tol)
    bar[list(truth_rows)] = 1e-3
    say(f"  relative gradient error: worst {rel[far].max():.2e} away from the truth"
        + (f", {rel[list(truth_rows)].max():.2e} at the truth" if len(truth_rows) else ""))
    worst = int(np.argmax(rel / bar))
    assert np.all(rel <= bar), (f"relative gradient error {rel[worst]:.3e} at point {worst} (bar {bar[worst]:.0e}): "
                                f"gpu {g[worst]} oracle {rg[worst]}")
    return rel


def small_spec(H=40, W=36, N=2, psf=None, pixscale=0.08, center=(0.05, -0.03)):
    base = mocks.c1_spec()
    psf = mocks.moffat_psf(7, 0.15, 3.0, pixscale) if psf is None else psf
    return mocks.SystemSpec(f"grad_{H}x{W}_sub{N}", H, W, N, psf.astype(np.float32), base.truth, base.prior,
                            mocks.annulus_mask(H, W, 0.2, 10.0, pixscale), 31, True, pixscale=pixscale,
                            center_x=center[0], center_y=center[1])


def small_obs(spec, seed=3):
    osys = oracle_system(spec)
    return mocks.make_observation(spec, lambda t: oracle.render(osys, np.asarray(t, np.float64)))


def test_gradient_small_system_random_points():
    spec = small_spec()
    say("gradient, 40x36 sub2, 24 prior points")
    obs = small_obs(spec)
    pts = mocks.points(spec, 24, seed=41)
    pts[0] = spec.truth
    check(spec, obs, pts, truth_rows=[0])


def test_gradient_when_the_signal_reaches_the_border():
    """Large PSF, source image near the edge: the replicate-padding fold of A^T matters."""
    psf = mocks.gaussian_psf(9, 0.3, 0.08) + 0.05
    spec = small_spec(H=24, W=20, N=3, psf=psf)
    say("gradient at the border fold")
    obs = small_obs(spec)
    pts = mocks.points(spec, 8, seed=43)
    pts[:, 0] = 0.6           # images near the edges of the 1.9" x 1.6" field
    pts[:, 10:12] = 0.15
    check(spec, obs, pts)


@pytest.mark.parametrize("H,W,P", [(1, 9, 5), (2, 11, 21), (9, 1, 5), (13, 2, 21), (3, 70, 21), (66, 3, 7)])
def test_gradient_on_degenerate_image_shapes(H, W, P):
    """Images one to three pixels high or wide: every pixel touches the border,
    the first and last rows (columns) coincide when H = 1 (W = 1), and the
    border segments of A^T rho are ragged (their window staged with zeros).
    With 8 to 208 weighted pixels the log L bar is not applied (one pixel's
    float32 error, within 1e-5 of the peak, moved log L by up to 3.3e-6 relative
    on the 13 x 2 image); the gradient bar is."""
    psf = mocks.moffat_psf(P, 0.3, 3.0, 0.2)
    spec = small_spec(H=H, W=W, N=2, psf=psf, pixscale=0.2, center=(0.1, -0.05))
    say(f"gradient, {H}x{W} sub2, {P}x{P} PSF")
    obs = small_obs(spec)
    pts = mocks.points(spec, 6, seed=59 + H + W)
    check(spec, obs, pts, loglike_bar=False)


def test_gradient_isothermal_sphere_and_round_source():
    spec = small_spec(H=32, W=32, N=4)
    say("gradient, q = 1 lens")
    obs = small_obs(spec)
    pts = mocks.points(spec, 6, seed=47)
    pts[:, 1] = 1.0           # SIS: derivative in q is the one-sided limit
    pts[3:, 15] = 1.0         # round source
    check(spec, obs, pts)


def test_gradient_wide_tiles_with_ragged_rows():
    """The 21x21 stencil on wide tiles (a whole row, or half of one) whose last
    row of tiles is ragged: the adjoint's A^T on those tiles."""
    psf = mocks.moffat_psf(21, 0.1, 3.0, 0.05)
    spec = small_spec(H=77, W=170, N=2, psf=psf, pixscale=0.05)
    say("gradient, 77x170 sub2, 21x21 PSF")
    obs = small_obs(spec)
    pts = mocks.points(spec, 6, seed=49)
    check(spec, obs, pts)


def test_gradient_full_c1_shape():
    """The C3 configuration: the 200x200 sub4 Moffat-21 model, 1024 points per launch;
    every 8th point (128, the truth first) against the oracle's exact gradient stored
    by tests/golden/make_golden.py."""
    spec, obs = observation("c1")
    say("gradient, C1 shape, 1024 points, 128 compared")
    pts = golden.c3_points(spec)
    gold = golden_file(golden.C3_FILE)
    assert str(gold["theta_sha256"]) == golden.digest(pts), "C3 points differ from those of the stored values"
    assert str(gold["data_sha256"]) == golden.digest(obs.data), "C1 mock differs from the stored one"
    assert str(gold["weight_sha256"]) == golden.digest(obs.weight)
    gsys = gpu_system(spec, obs)
    ll, g = lensed.loglike_grad(torch.from_numpy(pts).to(DEV), gsys)
    ll, g = ll.cpu().numpy(), g.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(g)) and np.all(np.isfinite(ll))
    idx = gold["index"]
    rll, rg = gold["loglike"], gold["grad"]
    lr = np.abs(ll[idx] - rll) / loglike_tolerance(rll, obs.weight)
    rel = np.linalg.norm(g[idx] - rg, axis=1) / np.linalg.norm(rg, axis=1)
    say(f"  worst |delta log L| / bar {lr.max():.3f}; gradient: truth {rel[0]:.2e}, "
        f"worst elsewhere {rel[1:].max():.2e} at point {int(idx[1 + np.argmax(rel[1:])])}")
    assert np.all(lr <= 1.0), lr.max()
    assert rel[0] <= 1e-3, rel[0]          # the truth: noise-driven gradient
    assert rel[1:].max() <= 1e-4, rel[1:].max()


def test_gradient_matches_oracle_central_differences():
    """Central differences of the FP64 oracle log L (Richardson-extrapolated), step
    h_j = 1e-4 max(|theta_j|, 0.01 x prior width_j)."""
    spec = small_spec(H=30, W=30, N=2)
    say("gradient vs oracle finite differences")
    obs = small_obs(spec)
    osys = oracle_system(spec, obs)
    t = spec.truth.astype(np.float32).copy()
    t[0] += 0.02; t[14] += 0.1; t[10] -= 0.01
    width = spec.prior.high - spec.prior.low
    gsys = gpu_system(spec, obs)
    _, g = lensed.loglike_grad(torch.from_numpy(t).view(1, 17).to(DEV), gsys)
    g = g.cpu().numpy()[0].astype(np.float64)
    tt = t.astype(np.float64)

    def fd(k):
        h = 1e-4 * max(abs(tt[k]), 0.01 * width[k])
        def f(dh):
            u = tt.copy(); u[k] += dh
            return oracle.loglike(osys, u)
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    with ThreadPoolExecutor(max_workers=8) as ex:
        ref = np.array(list(ex.map(fd, range(17))))
    assert np.linalg.norm(g - ref) <= 1e-4 * np.linalg.norm(ref), (g, ref)


def test_autograd_function_backward():
    spec = small_spec()
    obs = small_obs(spec)
    gsys = gpu_system(spec, obs)
    pts = torch.from_numpy(mocks.points(spec, 5, seed=53)).to(DEV).requires_grad_(True)
    ll = lensed.LogLikeFn.apply(pts, gsys)
    w = torch.linspace(0.5, 1.5, 5, device=DEV, dtype=torch.float64)
    (ll * w).sum().backward()
    _, g = lensed.loglike_grad(pts.detach(), gsys)
    assert torch.allclose(pts.grad, (w[:, None].float() * g), rtol=1e-6, atol=0)



def grad_into(ctx, theta, system, ll, g):
    """lensed_loglike_grad through the C ABI into fixed output buffers, so that
    calls with the same buffers reuse the context's cached plan."""
    import ctypes
    from paper_1505_07674_amd.binding import _stream_handle, lib
    rc = lib().lensed_loglike_grad(ctx.handle, ctypes.byref(system.c_struct), ctypes.c_void_p(theta.data_ptr()),
                                   theta.shape[0], ctypes.c_void_p(ll.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                   _stream_handle(None))
    ctx.check(rc, "lensed_loglike_grad")
    torch.cuda.synchronize()
    return ll.cpu().numpy().copy(), g.cpu().numpy().copy()


def test_gradient_follows_weights_changed_in_place():
    """The gradient kernels visit only the pixels within the PSF box of a w > 0
    pixel, a support rebuilt from the weights by every launch: a cached plan
    whose weights the caller changes in place (same pointers, same plan) must
    give what a fresh context gives, when the support grows and when it
    shrinks, and the oracle's gradient of the new data."""
    from paper_1505_07674_amd.binding import Context
    spec = small_spec(H=40, W=36, N=2)
    obs = small_obs(spec)
    pts = mocks.points(spec, 8, seed=43)
    tp = torch.from_numpy(pts).to(DEV)
    gs = gpu_system(spec, obs)
    full = gs.weight.clone()
    ll_buf = torch.empty(len(pts), dtype=torch.float64, device=DEV)
    g_buf = torch.empty((len(pts), 17), dtype=torch.float32, device=DEV)
    ctx = Context(0)
    results = []
    for label, cut in (("left half masked", slice(0, 18)), ("all weights", None), ("right third masked", slice(24, 36))):
        gs.weight.copy_(full)
        if cut is not None:
            gs.weight[:, cut] = 0.0
        say(f"weights in place: {label}")
        ll, g = grad_into(ctx, tp, gs, ll_buf, g_buf)
        fresh = Context(0)
        ll_f, g_f = grad_into(fresh, tp, gs, torch.empty_like(ll_buf), torch.empty_like(g_buf))
        fresh.close()
        assert np.array_equal(ll, ll_f), label
        assert np.array_equal(g, g_f), label
        results.append((label, gs.weight.cpu().numpy().copy(), g))
    ctx.close()
    for label, w, g in results[::2]:   # the two masked states against the oracle
        osys = oracle_system(spec, mocks.Observation(spec, obs.data, w, obs.sigma))
        _, ref = oracle_grads(osys, pts)
        rel = np.linalg.norm(g - ref, axis=1) / np.linalg.norm(ref, axis=1)
        say(f"  {label}: worst relative gradient error {rel.max():.2e}")
        assert np.all(rel <= 1e-4), (label, rel)


def test_gradient_plan_reused_after_an_invalid_point():
    """A gradient plan renders only the support of g and zeroes the rest of each
    image per launch, so a NaN point in one call (its image and g are NaN)
    leaves nothing behind for the valid point that takes its slot next."""
    from paper_1505_07674_amd.binding import Context
    spec = small_spec(H=40, W=36, N=2)
    obs = small_obs(spec)
    pts = mocks.points(spec, 6, seed=44)
    gs = gpu_system(spec, obs)
    gs.weight[:, 0:14] = 0.0   # a support well inside the image
    tp = torch.from_numpy(pts).to(DEV)
    slot = tp.clone()
    slot[2, 0] = float("nan")
    ll_buf = torch.empty(len(pts), dtype=torch.float64, device=DEV)
    g_buf = torch.empty((len(pts), 17), dtype=torch.float32, device=DEV)
    ctx = Context(0)
    ll_bad, _ = grad_into(ctx, slot, gs, ll_buf, g_buf)
    assert np.isnan(ll_bad[2]) and np.all(np.isfinite(ll_bad[[0, 1, 3, 4, 5]]))
    slot.copy_(tp)   # same buffers, same plan
    ll, g = grad_into(ctx, slot, gs, ll_buf, g_buf)
    ctx.close()
    fresh = Context(0)
    ll_f, g_f = grad_into(fresh, tp, gs, torch.empty_like(ll_buf), torch.empty_like(g_buf))
    fresh.close()
    say(f"after a NaN point: log L {ll[2]:.6g} (fresh {ll_f[2]:.6g})")
    assert np.array_equal(ll, ll_f)
    assert np.array_equal(g, g_f)
