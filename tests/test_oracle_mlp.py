"""Pins of the FP64 reference network (oracle/mlp.py): the forward pass and the
loss gradient against torch's own float64 layers (torch.nn.functional.linear
and silu, autograd), gradient against central differences, SiLU derivative,
bfloat16 rounding against torch's conversion, and the Adam update against its
closed-form first step and a convex problem."""
import numpy as np
import pytest
import torch

from oracle import mlp

RNG = np.random.default_rng(5)


def test_parameter_count():
    assert mlp.NPARAM == 136449


def test_bf16_rounding_matches_torch():
    x = np.concatenate([RNG.standard_normal(10000) * 10.0 ** RNG.uniform(-8, 8, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0, 3.0e38]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_silu_derivative():
    z = np.linspace(-8, 8, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.allclose(mlp.dsilu(z), fd, rtol=1e-8, atol=1e-10)


def _problem(B=64):
    theta = mlp.init_params(3).astype(np.float64)
    norm = np.concatenate([RNG.uniform(-1, 1, 17), RNG.uniform(0.5, 2, 17), [3.0, 2.0]])
    x = RNG.uniform(-1, 1, (B, 17))
    y = np.sin(x.sum(1)) * 2 + 3
    return theta, norm, x, y


def test_gradient_matches_central_differences():
    theta, norm, x, y = _problem()
    _, g = mlp.loss_and_grad(theta, norm, x, y, emulate_bf16=False)
    idx = np.concatenate([RNG.choice(17 * 256, 6, replace=False),                 # W1
                          [4352 + 7, 4352 + 256 + 1000, 136449 - 5, 136448],       # b1, W2, W4, b4
                          RNG.choice(mlp.NPARAM, 8, replace=False)])
    for i in idx:
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h; tm[i] -= h
        fd = (mlp.loss_and_grad(tp, norm, x, y, False)[0] - mlp.loss_and_grad(tm, norm, x, y, False)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_forward_output_units():
    theta, norm, x, y = _problem()
    out = mlp.forward(theta, norm, x, emulate_bf16=False)
    loss, _ = mlp.loss_and_grad(theta, norm, x, y, emulate_bf16=False)
    assert loss == pytest.approx(np.mean(((out - norm[34]) / norm[35] - (y - norm[34]) / norm[35]) ** 2), rel=1e-12)


def test_adam_first_step_and_convergence():
    g = RNG.standard_normal(50)
    th, m, v = mlp.adam_step(np.zeros(50), g, np.zeros(50), np.zeros(50), 1, lr=0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    target = RNG.standard_normal(50)
    th, m, v = np.zeros(50), np.zeros(50), np.zeros(50)
    for t in range(1, 3001):
        th, m, v = mlp.adam_step(th, th - target, m, v, t, lr=0.01)
    assert np.max(np.abs(th - target)) < 1e-3


def _torch_net(theta, norm):
    """The same network from torch's float64 layers: linear, silu, linear, silu,
    linear, silu, linear, with the input and output normalisation."""
    Ws, bs = mlp.unflatten(theta)
    P = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for pair in zip(Ws, bs) for a in pair]
    nt = torch.tensor(norm, dtype=torch.float64)
    F = torch.nn.functional

    def net(x):
        h = (torch.as_tensor(x, dtype=torch.float64) - nt[:17]) * nt[17:34]
        for l in range(3):
            h = F.silu(F.linear(h, P[2 * l], P[2 * l + 1]))
        return F.linear(h, P[6], P[7])[:, 0]
    return net, P, nt


def test_forward_matches_torch_layers():
    theta, norm, x, _ = _problem(B=200)
    theta = theta + 0.3 * RNG.standard_normal(theta.size)       # non-zero biases too
    net, _, nt = _torch_net(theta, norm)
    ref = (nt[34] + nt[35] * net(x)).detach().numpy()
    out = mlp.forward(theta, norm, x, emulate_bf16=False)
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-12 * np.max(np.abs(ref)))
    # a dropped bias, a transposed weight or a missing activation would not match
    assert np.max(np.abs(out - ref)) < 1e-9 * np.max(np.abs(ref))


def test_loss_gradient_matches_torch_autograd():
    theta, norm, x, y = _problem(B=96)
    theta = theta + 0.1 * RNG.standard_normal(theta.size)
    net, P, nt = _torch_net(theta, norm)
    t = (torch.tensor(y, dtype=torch.float64) - nt[34]) / nt[35]
    loss_t = torch.mean((net(x) - t) ** 2)
    loss_t.backward()
    gref = np.concatenate([p.grad.numpy().reshape(-1) for p in P])
    loss, g = mlp.loss_and_grad(theta, norm, x, y, emulate_bf16=False)
    assert loss == pytest.approx(loss_t.item(), rel=1e-12)
    assert np.allclose(g, gref, rtol=1e-9, atol=1e-12 * np.max(np.abs(gref)))
