"""Nested sampler on analytic problems (CPU): evidence of a Gaussian in the unit
box and of a two-mode mixture against their closed forms, posterior moments,
bitwise checkpoint/resume, and the screen (a perfect one saves exact calls, a
useless one cannot bias the result)."""
import math

import numpy as np
import pytest

from paper_1505_07674_amd.sampler import NestedSampler, Screen

D, MU, SIG = 4, 0.45, 0.04


def gauss(u):
    return -0.5 * np.sum(((u - MU) / SIG) ** 2, axis=1)


LOGZ_GAUSS = D * math.log(SIG * math.sqrt(2 * math.pi))


def test_gaussian_in_box_evidence_and_moments():
    res = NestedSampler(gauss, D, n_live=300, k_replace=20, seed=1).run()
    assert abs(res.logz - LOGZ_GAUSS) < 3 * res.logz_err + 0.05
    mean, std = res.posterior_moments(lambda u: u)
    assert np.allclose(mean, MU, atol=3 * SIG / math.sqrt(300))
    assert np.allclose(std, SIG, rtol=0.15)


def test_bimodal_mixture_evidence():
    c1, c2, s = 0.3, 0.7, 0.03

    def ll(u):
        a = -0.5 * np.sum(((u - c1) / s) ** 2, axis=1)
        b = -0.5 * np.sum(((u - c2) / s) ** 2, axis=1) + math.log(0.5)
        return np.logaddexp(a, b)
    d = 2
    truth = d * math.log(s * math.sqrt(2 * math.pi)) + math.log(1.5)
    res = NestedSampler(ll, d, n_live=400, k_replace=10, seed=3).run()
    assert abs(res.logz - truth) < 3 * res.logz_err + 0.05
    # both modes carry their share of the posterior mass
    w1 = res.weights[res.samples[:, 0] < 0.5].sum()
    assert w1 == pytest.approx(1 / 1.5, abs=0.08)


def test_checkpoint_resume_is_bitwise():
    a = NestedSampler(gauss, D, n_live=100, k_replace=10, seed=7)
    full = a.run()
    b = NestedSampler(gauss, D, n_live=100, k_replace=10, seed=7)
    b.run(max_iter=15)
    blob = b.checkpoint()
    c = NestedSampler(gauss, D, n_live=100, k_replace=10, seed=999)
    c.restore(blob)
    resumed = c.run()
    assert resumed.logz == full.logz
    assert np.array_equal(resumed.samples, full.samples)
    assert resumed.n_exact == full.n_exact


def test_perfect_screen_saves_exact_calls_without_changing_the_answer():
    plain = NestedSampler(gauss, D, n_live=200, k_replace=20, seed=5).run()
    screened = NestedSampler(gauss, D, n_live=200, k_replace=20, seed=5).run(
        screen=Screen(predict=gauss, margin=lambda lmin: 1e-9))
    assert screened.renders_per_accepted < 0.7 * plain.renders_per_accepted
    assert screened.renders_per_accepted < 1.5
    assert abs(screened.logz - LOGZ_GAUSS) < 3 * screened.logz_err + 0.05
    m1, _ = plain.posterior_moments(lambda u: u)
    m2, _ = screened.posterior_moments(lambda u: u)
    assert np.allclose(m1, m2, atol=0.2 * SIG)


def test_useless_screen_cannot_bias_the_result():
    """A screen that rejects everything falls back to exact batches; every accepted
    point is still exact, so the evidence stays right."""
    res = NestedSampler(gauss, D, n_live=200, k_replace=20, seed=6).run(
        screen=Screen(predict=lambda u: np.full(len(u), -1e30), margin=lambda lmin: 0.0, max_skips=50))
    assert abs(res.logz - LOGZ_GAUSS) < 3 * res.logz_err + 0.05


def test_multi_ellipsoid_bound_on_two_far_modes():
    """Two modes in 8 dimensions: the union of ellipsoids (recursive 2-means
    splits) draws ~4x fewer rejected candidates than one ellipsoid, and both give
    the closed-form evidence and equal mode weights."""
    d, s = 8, 0.02
    c1, c2 = np.full(d, 0.3), np.full(d, 0.7)

    def ll(u):
        return np.logaddexp(-0.5 * np.sum(((u - c1) / s) ** 2, axis=1), -0.5 * np.sum(((u - c2) / s) ** 2, axis=1))
    truth = d * math.log(s * math.sqrt(2 * math.pi)) + math.log(2)
    one = NestedSampler(ll, d, n_live=400, k_replace=20, seed=2, multi=False).run()
    many = NestedSampler(ll, d, n_live=400, k_replace=20, seed=2, multi=True).run()
    for r in (one, many):
        assert abs(r.logz - truth) < 3 * r.logz_err + 0.05
        assert r.weights[r.samples[:, 0] < 0.5].sum() == pytest.approx(0.5, abs=0.08)
    assert many.renders_per_accepted < 0.4 * one.renders_per_accepted


def test_audit_counts_false_rejections_of_a_biased_screen():
    """A screen that underestimates log L by a fixed 3 nats with no margin rejects
    good draws; auditing every screened-out draw exactly finds them, while the
    audit leaves the run itself (draws, acceptances, evidence) unchanged."""
    biased = Screen(predict=lambda u: gauss(u) - 3.0, margin=lambda lmin: 0.0)
    a = NestedSampler(gauss, D, n_live=150, k_replace=15, seed=9).run(screen=biased)
    b = NestedSampler(gauss, D, n_live=150, k_replace=15, seed=9, audit=1.0).run(screen=biased)
    assert a.n_audit == 0 and b.n_audit == b.n_screened_out > 0
    assert b.n_false_reject > 0
    assert b.logz == a.logz and b.n_exact == a.n_exact


def test_slice_replacements_give_the_gaussian_evidence_and_moments():
    """Slice-sampling chains (one per replacement, whitened random directions,
    n_steps = d slices each) instead of bounded rejection: same closed-form
    evidence and moments on a narrow 10-D Gaussian."""
    d, mu, sig = 10, np.linspace(0.35, 0.65, 10), 0.01
    ll = lambda u: -0.5 * np.sum(((u - mu) / sig) ** 2, axis=1)
    truth = d * math.log(sig * math.sqrt(2 * math.pi))
    r = NestedSampler(ll, d, n_live=300, k_replace=30, seed=11, method="slice").run()
    assert abs(r.logz - truth) < 3 * r.logz_err + 0.05
    mean, std = r.posterior_moments(lambda u: u)
    assert np.allclose(mean, mu, atol=4 * sig / math.sqrt(300))
    assert np.allclose(std, sig, rtol=0.15)


def test_screen_decides_slice_membership_without_changing_the_chains():
    """With a screen that predicts log L to within the margin, every membership
    decision it takes is the exact one, so the slice chains, the evidence and the
    samples are those of the unscreened run, with several times fewer exact
    evaluations; an audit of the screen's decisions finds no false rejection."""
    d, mu, sig = 10, np.linspace(0.35, 0.65, 10), 0.01
    ll = lambda u: -0.5 * np.sum(((u - mu) / sig) ** 2, axis=1)
    noisy = lambda u: ll(u) + np.random.default_rng(len(u)).uniform(-0.9, 0.9, len(u))
    plain = NestedSampler(ll, d, n_live=200, k_replace=20, seed=12, method="slice").run()
    scr = NestedSampler(ll, d, n_live=200, k_replace=20, seed=12, method="slice", audit=0.05).run(
        screen=Screen(predict=noisy, margin=lambda lmin: 1.0))
    assert scr.logz == plain.logz and np.array_equal(scr.samples, plain.samples)
    assert scr.renders_per_accepted < 0.35 * plain.renders_per_accepted
    assert scr.n_audit > 1000 and scr.n_false_reject == 0
