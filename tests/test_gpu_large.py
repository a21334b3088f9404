"""Launches past the hardware's per-dimension grid limits: item lists longer
than one launch can hold are split (render, PSF, adjoint) and the adjoint's
border pass covers more than 65535 points. The per-point results equal those
of small batches of the same points."""
import numpy as np
import pytest
import torch

import paper_1505_07674_amd as lensed
from paper_1505_07674_amd import mocks

from helpers import observation

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def c0_system():
    spec, obs = observation("c0")
    return spec, lensed.System(torch.from_numpy(spec.psf).to(DEV), torch.from_numpy(obs.data).to(DEV),
                               torch.from_numpy(obs.weight).to(DEV), pixscale=spec.pixscale, nsub=spec.nsub)


def test_batch_longer_than_one_launch():
    """270 000 C0 points: 16 render tiles each, 4.3 M render blocks, more than
    one launch takes (2^22)."""
    spec, g = c0_system()
    n = 270_000
    pts = mocks.points(spec, n, seed=71).astype(np.float32)
    tp = torch.from_numpy(pts).to(DEV)
    say(f"c0 loglike batch, {n} points")
    big = lensed.loglike_batch(tp, np.zeros(n, np.int32), [g]).cpu().numpy()
    assert np.all(np.isfinite(big))
    idx = np.concatenate([np.arange(0, 64), np.arange(n - 64, n), np.arange(4_194_304 // 16 - 32, 4_194_304 // 16 + 32)])
    small = lensed.loglike_batch(tp[idx].contiguous(), np.zeros(len(idx), np.int32), [g]).cpu().numpy()
    assert np.array_equal(big[idx], small)
    del tp
    torch.cuda.empty_cache()


def test_gradient_over_more_than_65535_points():
    spec, g = c0_system()
    n = 66_000
    pts = mocks.points(spec, n, seed=72).astype(np.float32)
    tp = torch.from_numpy(pts).to(DEV)
    say(f"c0 gradient, {n} points")
    ll, gr = lensed.loglike_grad(tp, g)
    gr = gr.cpu().numpy()
    assert np.all(np.isfinite(gr))
    idx = np.concatenate([np.arange(0, 16), np.arange(65_520, 65_552), np.arange(n - 16, n)])
    ll2, gr2 = lensed.loglike_grad(tp[idx].contiguous(), g)
    assert np.array_equal(gr[idx], gr2.cpu().numpy())
    assert np.array_equal(ll.cpu().numpy()[idx], ll2.cpu().numpy())
    del tp
    torch.cuda.empty_cache()
