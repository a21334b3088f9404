"""GPU surrogate-network kernels (bfloat16 MFMA, float32 accumulation) against
the FP64 reference network fed the same bfloat16-rounded operands.

Bars: forward ||y_gpu - y_ref|| <= 1e-2 ||y_ref - mean(y_ref)||; loss within
1e-3 relative; every gradient tensor (W1..b4) within 1e-2 of the reference
tensor's norm; Adam within 1e-5 relative of the reference update.
"""
import numpy as np
import pytest
import torch

import paper_1505_07674_amd as lensed
from oracle import mlp as ref

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
RNG = np.random.default_rng(11)
NAMES = ["W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4"]


def problem(B):
    theta = ref.init_params(7)
    theta[ref.LAYERS[1] * 17:ref.LAYERS[1] * 17 + 256] = RNG.uniform(-0.1, 0.1, 256)   # non-zero b1
    norm = np.concatenate([RNG.uniform(-1, 1, 17), RNG.uniform(0.5, 2, 17), [-5.0, 3.0]]).astype(np.float32)
    x = RNG.uniform(-1.5, 1.5, (B, 17)).astype(np.float32)
    y = (np.sin(x.sum(1)) * 3.0 - 5.0 + 0.3 * x[:, 0] ** 2).astype(np.float32)
    return theta.astype(np.float32), norm, x, y


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("B", [1, 97, 777])
def test_forward_matches_reference(B):
    theta, norm, x, _ = problem(B)
    y = lensed.mlp_forward(dev(theta), dev(norm), dev(x)).cpu().numpy().astype(np.float64)
    yr = ref.forward(theta, norm, x, emulate_bf16=True)
    scale = np.linalg.norm(yr - yr.mean()) if B > 1 else abs(yr[0] - norm[34]) + 1.0
    assert np.linalg.norm(y - yr) <= 1e-2 * scale


@pytest.mark.parametrize("B", [64, 300])
def test_gradient_matches_reference(B):
    theta, norm, x, y = problem(B)
    loss, g = lensed.mlp_grad(dev(theta), dev(norm), dev(x), dev(y))
    lr_, gr = ref.loss_and_grad(theta, norm, x, y, emulate_bf16=True)
    assert float(loss.cpu()) == pytest.approx(lr_, rel=1e-3)
    g = g.cpu().numpy().astype(np.float64)
    Wg, bg = ref.unflatten(g)
    Wr, br = ref.unflatten(gr)
    for name, a, b in zip(NAMES, [t for pair in zip(Wg, bg) for t in pair], [t for pair in zip(Wr, br) for t in pair]):
        assert np.linalg.norm(a - b) <= 1e-2 * np.linalg.norm(b), name


def test_adam_matches_reference():
    theta, _, _, _ = problem(8)
    g = RNG.standard_normal(ref.NPARAM).astype(np.float32)
    m = (RNG.standard_normal(ref.NPARAM) * 0.1).astype(np.float32)
    v = (RNG.random(ref.NPARAM) * 0.1).astype(np.float32)
    tp, tm, tv = dev(theta), dev(m), dev(v)
    lensed.mlp_adam(tp, dev(g), tm, tv, 3, 1e-3)
    er, em, ev = ref.adam_step(theta.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                               v.astype(np.float64), 3, 1e-3)
    assert np.allclose(tm.cpu().numpy(), em, rtol=1e-5, atol=1e-7)
    assert np.allclose(tv.cpu().numpy(), ev, rtol=1e-5, atol=1e-9)
    assert np.allclose(tp.cpu().numpy(), er, rtol=1e-5, atol=1e-7)


def test_training_reduces_the_loss():
    theta, norm, x, y = problem(2048)
    p, m, v = dev(theta), torch.zeros(ref.NPARAM, device=DEV), torch.zeros(ref.NPARAM, device=DEV)
    X, Y = dev(x), dev(y)
    first = None
    for step in range(1, 301):
        i = (step - 1) % 8
        loss = lensed.mlp_train_step(p, m, v, step, dev(norm), X[i * 256:(i + 1) * 256], Y[i * 256:(i + 1) * 256],
                                     1e-3)
        if first is None:
            first = float(loss.cpu())
    final = float(lensed.mlp_grad(p, dev(norm), X, Y)[0].cpu())
    assert final < 0.15 * first, (first, final)


def test_training_tracks_the_reference_optimiser():
    """40 Adam steps on the GPU and in the FP64 reference (same mini-batches, same
    bfloat16 rounding points) reach the same full-batch loss within 10 %."""
    theta, norm, x, y = problem(1024)
    p, m, v = dev(theta), torch.zeros(ref.NPARAM, device=DEV), torch.zeros(ref.NPARAM, device=DEV)
    X, Y = dev(x), dev(y)
    rp, rm, rv = theta.astype(np.float64), np.zeros(ref.NPARAM), np.zeros(ref.NPARAM)
    for step in range(1, 41):
        i = (step - 1) % 4
        sl = slice(i * 256, (i + 1) * 256)
        lensed.mlp_train_step(p, m, v, step, dev(norm), X[sl], Y[sl], 2e-3)
        _, g = ref.loss_and_grad(rp, norm, x[sl], y[sl], emulate_bf16=True)
        rp, rm, rv = ref.adam_step(rp, g, rm, rv, step, 2e-3)
    l_gpu = ref.loss_and_grad(p.cpu().numpy().astype(np.float64), norm, x, y, emulate_bf16=True)[0]
    l_ref = ref.loss_and_grad(rp, norm, x, y, emulate_bf16=True)[0]
    l0 = ref.loss_and_grad(theta.astype(np.float64), norm, x, y, emulate_bf16=True)[0]
    assert l_ref < 0.5 * l0, (l0, l_ref)
    assert abs(l_gpu - l_ref) <= 0.1 * l_ref, (l0, l_gpu, l_ref)
