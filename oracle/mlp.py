"""FP64 reference of the surrogate network -- TEST INFRASTRUCTURE ONLY.

A multilayer perceptron 17 -> 256 -> 256 -> 256 -> 1 with SiLU activations,
z * sigmoid(z), trained on mean squared error with Adam (Kingma & Ba 2015). It
is the plain definition written out with numpy matrix products, used to check
the GPU kernels. Only the tests may import it.

With ``emulate_bf16`` the operands are rounded to bfloat16 (round to nearest
even) exactly where the GPU kernels feed their matrix cores: the normalised
input, the weights, the activations H and the back-propagated dZ. Every sum is
taken in float64; everything else (biases, pre-activations, the head GEMV and
the loss) stays in float64.

Flat parameter layout (136449 values): W1 [256][17], b1 [256], W2 [256][256],
b2 [256], W3 [256][256], b3 [256], W4 [1][256], b4 [1].
Normalisation block (36 values): x_shift [17], x_scale [17], y_shift, y_scale;
the network sees (x - x_shift) * x_scale and predicts (y - y_shift) / y_scale.
"""
import numpy as np

LAYERS = (17, 256, 256, 256, 1)
NPARAM = sum(LAYERS[i] * LAYERS[i + 1] + LAYERS[i + 1] for i in range(len(LAYERS) - 1))


def bf16(x):
    """Round float values to bfloat16 (nearest, ties to even) and return float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    out = np.where(nan, a, out)
    return out.astype(np.float64)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def unflatten(theta):
    theta = np.asarray(theta, dtype=np.float64).reshape(-1)
    assert theta.size == NPARAM
    Ws, bs, o = [], [], 0
    for i in range(len(LAYERS) - 1):
        n_in, n_out = LAYERS[i], LAYERS[i + 1]
        Ws.append(theta[o:o + n_in * n_out].reshape(n_out, n_in)); o += n_in * n_out
        bs.append(theta[o:o + n_out]); o += n_out
    return Ws, bs


def flatten(Ws, bs):
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in zip(Ws, bs)])


def init_params(seed):
    """He-style uniform initialisation (float32 values)."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for i in range(len(LAYERS) - 1):
        n_in, n_out = LAYERS[i], LAYERS[i + 1]
        lim = np.sqrt(6.0 / n_in) if i < len(LAYERS) - 2 else np.sqrt(1.0 / n_in)
        Ws.append(rng.uniform(-lim, lim, size=(n_out, n_in)))
        bs.append(np.zeros(n_out))
    return flatten(Ws, bs).astype(np.float32)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(theta, norm, x, emulate_bf16=True, cache=False):
    """Network output in target units: y_shift + y_scale * net((x - x_shift) * x_scale)."""
    Ws, bs = unflatten(theta)
    norm = np.asarray(norm, dtype=np.float64)
    xs, xc, ys, yc = norm[:17], norm[17:34], norm[34], norm[35]
    h = _r((np.asarray(x, np.float64) - xs) * xc, emulate_bf16)
    hs, zs = [h], []
    for l in range(3):
        z = h @ _r(Ws[l], emulate_bf16).T + bs[l]
        h = _r(silu(z), emulate_bf16)
        zs.append(z)
        hs.append(h)
    out = (h @ _r(Ws[3], emulate_bf16).T)[:, 0] + bs[3][0]
    y = ys + yc * out
    if cache:
        return y, (out, hs, zs)
    return y


def loss_and_grad(theta, norm, x, y, emulate_bf16=True):
    """Mean squared error in normalised target units and its gradient (flat)."""
    Ws, bs = unflatten(theta)
    norm = np.asarray(norm, dtype=np.float64)
    ys, yc = norm[34], norm[35]
    _, (out, hs, zs) = forward(theta, norm, x, emulate_bf16, cache=True)
    t = (np.asarray(y, np.float64) - ys) / yc
    B = len(t)
    loss = np.mean((out - t) ** 2)
    d = 2.0 * (out - t) / B                           # d loss / d out
    gW = [None] * 4
    gb = [None] * 4
    gW[3] = (d @ hs[3])[None, :]
    gb[3] = np.array([d.sum()])
    dh = np.outer(d, _r(Ws[3], emulate_bf16)[0])      # d loss / d H3
    for l in (2, 1, 0):
        dz = dh * dsilu(zs[l])
        gb[l] = dz.sum(axis=0)
        dzr = _r(dz, emulate_bf16)
        gW[l] = dzr.T @ hs[l]
        if l > 0:
            dh = dzr @ _r(Ws[l], emulate_bf16)
    return loss, flatten(gW, gb)


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
