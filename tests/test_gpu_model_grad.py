"""GPU adjoint of general models (lensed_loglike_model_grad; Sec. 5: several
SIEs with free centres, the shear, several Sersic components, the sky; lenses
on several planes, Sec. 6) against Richardson-extrapolated central differences
of the FP64 oracle's log L, on the base model against the 17-parameter
adjoint, and with coincident planes against the one-plane adjoint.

Bar (per point, away from the truth of the mock): ||g_gpu - g_ref||_2 <= 1e-4
||g_ref||_2, the bar of the 17-parameter adjoint; the log L it returns equals
the batched general-model log L of the same points. The oracle has no
derivative of general models, so the reference is the finite-difference
gradient: steps h_k = 1e-4 max(|theta_k|, 0.05), two step sizes combined to
cancel the h^2 term."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import paper_1505_07674_amd as lensed
from paper_1505_07674_amd import mocks

from test_gpu_grad import small_spec
from test_gpu_model import PLANES_41, companion_points, gsys, models, osys

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def fd_grad(o, om, t):
    tt = np.asarray(t, np.float64)

    def one(k):
        h = 1e-4 * max(abs(tt[k]), 0.05)

        def f(dh):
            u = tt.copy()
            u[k] += dh
            return oracle.loglike_model(o, om, u)
        d1 = (f(h) - f(-h)) / (2 * h)
        d2 = (f(h / 2) - f(-h / 2)) / h
        return (4 * d2 - d1) / 3

    with ThreadPoolExecutor(max_workers=8) as ex:
        return np.array(list(ex.map(one, range(len(tt)))))


def mock(spec, om, truth, rule=None):
    model = oracle.render_model(osys(spec, rule=rule), om, truth.astype(np.float64))
    sigma = 0.01 * model.max()
    data = (model + sigma * np.random.default_rng(spec.width).standard_normal(model.shape)).astype(np.float32)
    weight = np.full(model.shape, 1.0 / sigma ** 2, np.float32)
    weight[:2, :] = 0.0    # a masked strip along the border
    return data, weight


@pytest.mark.parametrize("rule", ["sub", "g3k7"])
def test_general_model_gradient_matches_oracle_differences(rule):
    spec = small_spec(H=40, W=36, N=2)
    gm, om = models(2, PLANES_41, sky=True)
    truth = companion_points(1, seed=71)[0]
    orule = None if rule == "sub" else rule
    data, weight = mock(spec, om, truth, orule)
    g = gsys(spec, data, weight, rule=rule)
    o = osys(spec, data.astype(np.float64), weight.astype(np.float64), rule=orule)
    pts = companion_points(3, seed=76)
    pts[0] = truth + np.float32(0.02) * np.sign(np.random.default_rng(1).standard_normal(41)).astype(np.float32)
    q_index = [3, 8, 17, 24, 31, 38]   # the axis ratios (of the SIEs and the Sersics) stay in (0, 1]
    pts[0, q_index] = truth[q_index]
    tp = torch.from_numpy(pts).to(DEV)
    say(f"general-model gradient (41 parameters), rule {rule}, 3 points")
    ll, gg = lensed.loglike_model_grad(tp, g, gm)
    lb = lensed.loglike_model_batch(tp, np.zeros(3, np.int32), [g], gm).cpu().numpy()
    ll, gg = ll.cpu().numpy(), gg.cpu().numpy().astype(np.float64)
    assert np.allclose(ll, lb, rtol=1e-12, atol=0)
    for i, t in enumerate(pts):
        ref = fd_grad(o, om, t)
        rel = np.linalg.norm(gg[i] - ref) / np.linalg.norm(ref)
        worst = int(np.argmax(np.abs(gg[i] - ref)))
        say(f"  point {i}: relative error {rel:.2e} (largest at parameter {worst}: {gg[i][worst]:.6g} vs "
            f"{ref[worst]:.6g})")
        assert rel <= 1e-4, (i, rel, gg[i], ref)


def test_base_model_gradient_matches_the_17_parameter_adjoint():
    spec = small_spec()
    gm, om = models(1, ["foreground", "lensed"])
    obs = mocks.make_observation(spec, lambda t: oracle.render(osys(spec), np.asarray(t, np.float64)))
    g = gsys(spec, obs.data, obs.weight)
    pts = mocks.points(spec, 6, seed=77).astype(np.float32)
    general = np.array([np.concatenate([[0.0, 0.0], t[0:3], t[3:5], [0.0, 0.0], t[5:10], t[10:17]]) for t in pts],
                       np.float32)
    say("base model: general-model adjoint against the 17-parameter adjoint, 6 points")
    _, g17 = lensed.loglike_grad(torch.from_numpy(pts).to(DEV), g)
    _, gmod = lensed.loglike_model_grad(torch.from_numpy(general).to(DEV), g, gm)
    g17, gmod = g17.cpu().numpy().astype(np.float64), gmod.cpu().numpy().astype(np.float64)
    keep = [2, 3, 4, 5, 6, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20]   # the 17 shared parameters, in order
    rel = np.linalg.norm(gmod[:, keep] - g17, axis=1) / np.linalg.norm(g17, axis=1)
    say(f"  relative difference: worst {rel.max():.2e}")
    assert np.all(rel <= 1e-4), rel


def test_gradient_with_coincident_planes_is_the_one_plane_gradient():
    """Two lens planes with every SIE on plane 0 and plane 1 empty bend rays as
    one plane does: the dual-number chain of the several-plane adjoint must give
    the one-plane adjoint's gradient (both float64 rays; the Sersic profiles'
    float32 fractions are evaluated in a different order, hence the 1e-5 bar)."""
    spec = small_spec(H=40, W=36, N=2)
    gm1, om1 = models(2, PLANES_41, sky=True)
    gm2 = lensed.Model(2, PLANES_41, shear=True, sky=True, sie_planes=[0, 0], beta=[[0.0, 0.6], [0.0, 0.0]])
    truth = companion_points(1, seed=71)[0]
    data, weight = mock(spec, om1, truth)
    g = gsys(spec, data, weight)
    pts = torch.from_numpy(companion_points(4, seed=78)).to(DEV)
    say("coincident planes: several-plane adjoint against the one-plane adjoint, 4 points")
    ll1, g1 = lensed.loglike_model_grad(pts, g, gm1)
    ll2, g2 = lensed.loglike_model_grad(pts, g, gm2)
    g1, g2 = g1.cpu().numpy().astype(np.float64), g2.cpu().numpy().astype(np.float64)
    assert np.allclose(ll1.cpu().numpy(), ll2.cpu().numpy(), rtol=1e-9, atol=0)
    rel = np.linalg.norm(g2 - g1, axis=1) / np.linalg.norm(g1, axis=1)
    say(f"  relative difference: worst {rel.max():.2e}")
    assert np.all(rel <= 1e-5), rel


@pytest.mark.parametrize("rule", ["sub", "g3k7"])
def test_three_plane_gradient_matches_oracle_differences(rule):
    """Three lens planes (46 parameters: 3 SIEs, the shear, 4 Sersics, a sky)
    against the oracle's log L differences."""
    from test_gpu_multiplane import models as plane_models, three_plane_points
    spec = small_spec(H=40, W=36, N=2)
    gm, om = plane_models()
    truth = three_plane_points(1, seed=81)[0]
    orule = None if rule == "sub" else rule
    data, weight = mock(spec, om, truth, orule)
    g = gsys(spec, data, weight, rule=rule)
    o = osys(spec, data.astype(np.float64), weight.astype(np.float64), rule=orule)
    pts = three_plane_points(2, seed=82)
    tp = torch.from_numpy(pts).to(DEV)
    say(f"three-plane gradient (46 parameters), rule {rule}, 2 points")
    ll, gg = lensed.loglike_model_grad(tp, g, gm)
    lb = lensed.loglike_model_batch(tp, np.zeros(2, np.int32), [g], gm).cpu().numpy()
    ll, gg = ll.cpu().numpy(), gg.cpu().numpy().astype(np.float64)
    assert np.allclose(ll, lb, rtol=1e-12, atol=0)
    for i, t in enumerate(pts):
        ref = fd_grad(o, om, t)
        rel = np.linalg.norm(gg[i] - ref) / np.linalg.norm(ref)
        worst = int(np.argmax(np.abs(gg[i] - ref)))
        say(f"  point {i}: relative error {rel:.2e} (largest at parameter {worst}: {gg[i][worst]:.6g} vs "
            f"{ref[worst]:.6g})")
        assert rel <= 1e-4, (i, rel, gg[i], ref)


def test_autograd_function_backward_is_the_adjoint():
    """LogLikeModelFn: torch's backward of sum(c * log L) is c times the adjoint's gradient."""
    spec = small_spec(H=40, W=36, N=2)
    gm, om = models(2, PLANES_41, sky=True)
    truth = companion_points(1, seed=71)[0]
    data, weight = mock(spec, om, truth)
    g = gsys(spec, data, weight)
    pts = torch.from_numpy(companion_points(3, seed=79)).to(DEV).requires_grad_(True)
    coef = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device=DEV)
    ll = lensed.LogLikeModelFn.apply(pts, g, gm)
    (coef * ll).sum().backward()
    _, ref = lensed.loglike_model_grad(pts.detach(), g, gm)
    assert torch.equal(pts.grad, coef.to(torch.float32)[:, None] * ref)
