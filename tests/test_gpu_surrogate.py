"""The learned screen end to end on the GPU: nested sampling on the 64x64 mock
with and without the surrogate network, which is trained on the plain run's
exact (theta, log L) pairs by the library's own kernels.

What the network gains over the method without it: exact renders per accepted
point drop by at least 2x at this small size (the 200x200 experiment is run by
``python -m paper_1505_07674_amd.screened``), while the posterior means move
by no more than the sampler's own seed-to-seed spread allows.
"""
import numpy as np
import pytest
import torch

from paper_1505_07674_amd import mocks
from paper_1505_07674_amd.screened import GpuLogLike, compare_runs
from paper_1505_07674_amd.surrogate import Surrogate

from helpers import observation

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def test_gpu_loglike_wrapper_pads_and_matches_direct_batch():
    spec, obs = observation("c0")
    ll = GpuLogLike(spec, obs, DEV)
    u = np.random.default_rng(3).random((100, len(ll.free)))
    a = ll(u)
    b = np.concatenate([ll(u[:37]), ll(u[37:])])
    assert a.shape == (100,) and np.all(np.isfinite(a))
    assert np.array_equal(a, b)
    assert ll.n_points == 200


def test_surrogate_fits_loglike_pairs():
    spec, obs = observation("c0")
    ll = GpuLogLike(spec, obs, DEV)
    rng = np.random.default_rng(5)
    u = rng.random((20000, len(ll.free)))
    y = ll(u)
    sur = Surrogate(DEV, seed=1, free=ll.free)
    say("fitting 20000 prior pairs")
    fit = sur.fit(u, y, epochs=20, batch=512)
    assert fit["final_loss"] < 0.05, fit
    assert fit["rmse_y"] < 0.2, fit


def test_screen_cuts_exact_renders_and_keeps_the_posterior():
    spec, obs = observation("c0")
    res = compare_runs(spec, obs, DEV, n_live=100, k_replace=10, seeds=(mocks.C4_SEED, mocks.C4_SEED + 1,
                                                                        mocks.C4_SEED + 2),
                       train_epochs=30, train_batch=512, log=say, log_every=100)
    say(f"renders/accepted plain {res['plain']['renders_per_accepted']:.2f} "
        f"screened {res['screened']['renders_per_accepted']:.2f}; max shift {res['max_shift_screened_sigma']:.3f} "
        f"sigma (null {res['max_shift_null_sigma']:.3f})")
    assert res["renders_per_accepted_ratio"] >= 2.0, res
    # every accepted point is exact, so only a biased screen could move the posterior
    assert res["max_shift_screened_sigma"] <= max(0.5, 2.0 * res["max_shift_null_sigma"]), res
    assert abs(res["screened"]["logz"] - res["plain"]["logz"]) <= 3 * np.hypot(res["plain"]["logz_err"],
                                                                              res["screened"]["logz_err"]) + 0.5
