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
