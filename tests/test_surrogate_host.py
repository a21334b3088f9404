"""Host-side logic of the surrogate (CPU): the feature-map change of a local
refit leaves the network's function of theta unchanged (checked with the FP64
reference network on the same parameters)."""
import numpy as np
import torch

from oracle import mlp as ref
from paper_1505_07674_amd.surrogate import Surrogate


def test_feature_map_change_preserves_the_network_function():
    free = np.array([0, 2, 3, 5, 8, 9, 12])
    s = Surrogate(torch.device("cpu"), seed=3, free=free)
    s._set_norm(1.5, 0.7)
    rng = np.random.default_rng(0)
    u = rng.random((64, len(free)))

    def out():
        x = s._x(u).numpy().astype(np.float64)
        return ref.forward(s.params.numpy().astype(np.float64), s.norm.numpy().astype(np.float64), x,
                           emulate_bf16=False)
    y0 = out()
    a = rng.standard_normal((len(free), len(free)))
    s._remap(rng.random(len(free)), a @ a.T + np.eye(len(free)))     # a correlated whitening
    y1 = out()
    s._remap(rng.random(len(free)) * 0.1, np.diag(rng.random(len(free)) * 100 + 1))
    y2 = out()
    scale = np.std(y0)
    assert np.max(np.abs(y1 - y0)) < 1e-5 * scale + 1e-7
    assert np.max(np.abs(y2 - y0)) < 1e-5 * scale + 1e-7


def test_fixed_parameters_enter_the_network_as_zero():
    free = np.array([1, 4])
    s = Surrogate(torch.device("cpu"), seed=1, free=free)
    x = s._x(np.array([[0.25, 0.75]])).numpy()
    assert x.shape == (1, 17)
    assert np.all(x[0, [i for i in range(17) if i not in (1, 4)]] == 0)
    assert np.allclose(x[0, [1, 4]], [-0.5, 0.5])       # unit cube onto [-1, 1]
