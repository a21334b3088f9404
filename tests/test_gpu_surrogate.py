"""The learned screen end to end on the GPU: nested sampling with and without
the surrogate network, which is trained on the plain run's exact (theta, log L)
pairs by the library's own kernels.

What the network gains over the method without it: exact renders per accepted
point drop by at least 2x over the first iterations of a short run on the
200x200 mock (the full runs with 400 live points and the posterior comparison
are made by ``python -m paper_1505_07674_amd.screened``), and an exact audit of
screened-out draws finds (almost) no draw the screen should have kept.
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


def test_screen_cuts_exact_renders_without_false_rejections():
    """The 200x200 SIE + shear + Sersic mock, 100 live points, the first 100
    iterations: the plain run's exact pairs train the network, and the screened
    run needs far fewer exact renders per accepted point. A fifth of the
    screened-out draws are also evaluated exactly (an audit that does not change
    the run): almost none of them would have been accepted."""
    spec, obs = observation("c1")
    res = compare_runs(spec, obs, DEV, n_live=100, k_replace=10, max_iter=100,
                       seeds=(mocks.C4_SEED, mocks.C4_SEED + 1, mocks.C4_SEED + 2), train_epochs=150,
                       train_batch=512, record_per_iter=None, audit=0.2, log=say, log_every=25)
    sc = res["screened"]
    say(f"renders/accepted plain {res['plain']['renders_per_accepted']:.2f} "
        f"screened {sc['renders_per_accepted']:.2f} (x{res['renders_per_accepted_ratio']:.2f}); "
        f"audit {sc['n_audit']} draws, {sc['n_false_reject']} false rejections, {sc['n_false_accept']} false "
        f"acceptances; fit {res['fit']}; plain {res['plain']}; screened {sc}")
    assert res["renders_per_accepted_ratio"] >= 2.0, res
    assert sc["n_audit"] > 100
    assert sc["n_false_reject"] + sc["n_false_accept"] <= max(2, 0.01 * sc["n_audit"]), sc
