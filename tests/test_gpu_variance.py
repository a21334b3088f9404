"""GPU parity of the variance estimate from the data (Sec. 3.3, Eqs. 18-21)
against the oracle: weights w = extra g / (d + b), zero where the counts are
not positive, with scalar and per-pixel gain and offset, an extra weight factor
that masks, ragged and empty sizes, and the argument checks of the C ABI."""
import numpy as np
import pytest
import torch

import paper_1505_07674_amd as lensed
from oracle.variance import weights_from_data as oracle_weights
from paper_1505_07674_amd.binding import LensedError

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(DEV)


def check(w_gpu, w_ref):
    w = w_gpu.cpu().numpy().astype(np.float64)
    ref = w_ref.astype(np.float32).astype(np.float64)        # both round float64 once to float32
    assert np.array_equal(w == 0, ref == 0)
    assert np.all(np.abs(w - ref) <= 2.0 ** -23 * np.abs(ref))


@pytest.mark.parametrize("shape", [(200, 200), (37, 53), (1, 1), (3, 100003)])
def test_weights_match_the_oracle(shape):
    rng = np.random.default_rng(sum(shape))
    d = rng.uniform(-0.3, 4.0, shape).astype(np.float32)
    g = rng.uniform(50.0, 5000.0, shape).astype(np.float32)
    b = rng.uniform(0.0, 0.5, shape).astype(np.float32)
    e = rng.uniform(0.0, 2.0, shape).astype(np.float32)
    e[rng.random(shape) < 0.1] = 0.0
    check(lensed.weights_from_data(gpu(d), gpu(g), gpu(b), gpu(e)), oracle_weights(d, g, b, e))
    check(lensed.weights_from_data(gpu(d), 1200.0, 0.25), oracle_weights(d, 1200.0, 0.25))
    check(lensed.weights_from_data(gpu(d), gpu(g), 0.0), oracle_weights(d, g, 0.0))
    check(lensed.weights_from_data(gpu(d), 900.0, gpu(b), gpu(e)), oracle_weights(d, 900.0, b, e))


def test_poisson_mock_weights_feed_the_likelihood():
    """Weights from a Poisson mock of a constant image: with the model equal to
    the noiseless image, -2 log L per pixel averages to about 1."""
    rng = np.random.default_rng(8)
    H = W = 64
    g, b, level = 2000.0, 0.1, 0.8
    k = rng.poisson((level + b) * g, (H, W))
    d = (k / g - b).astype(np.float32)
    w = lensed.weights_from_data(gpu(d), g, b)
    sysm = lensed.System(gpu(np.ones((1, 1))), gpu(d), w, pixscale=0.05, nsub=1)
    theta = np.zeros(17, np.float32)
    theta[[1, 6, 7, 8, 13, 14, 15]] = [1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0]
    theta[5] = 0.0                                  # no lens light
    theta[12] = 0.0                                  # no source: the model is 0
    model0 = float(lensed.loglike(gpu(theta), sysm).cpu())
    chi2_ref = float(np.sum(oracle_weights(d, g, b).astype(np.float32) * d.astype(np.float64) ** 2))
    assert abs(-2 * model0 - chi2_ref) <= 1e-6 * chi2_ref
    mean_chi2 = float(np.mean(oracle_weights(d, g, b) * (d - level) ** 2))
    assert abs(mean_chi2 - 1.0) < 0.1


def test_empty_and_invalid_arguments():
    out = lensed.weights_from_data(torch.empty(0, device=DEV), 10.0)
    assert out.numel() == 0
    d = gpu(np.ones(5))
    for gain in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(LensedError):
            lensed.weights_from_data(d, gain)
    with pytest.raises(LensedError):
        lensed.weights_from_data(d, 1.0, float("nan"))
    with pytest.raises(ValueError):
        lensed.weights_from_data(d, gpu(np.ones(4)))
