"""Per-pixel weights estimated from the data -- TEST INFRASTRUCTURE ONLY.

Sec. 3.3 (Eqs. 18-21): with an effective gain g_i (data units -> photon counts)
and an offset b_i that was subtracted from the data (e.g. the sky), the counts
are k_i = g_i (d_i + b_i) (Eq. 18); taking them as Poisson, Var(k_i) = k_i
(Eq. 20), so the data variance is s_i^2 = Var(k_i) / g_i^2 = (d_i + b_i) / g_i
(Eq. 21). The paper adds an optional multiplicative extra weight factor; the
weight of a pixel is w_i = extra_i / s_i^2, and an extra factor of 0 masks it.

Reading: where the counts are not positive (k_i <= 0) the Poisson estimate has no
meaning and the pixel gets weight 0.
"""
import numpy as np


def weights_from_data(data, gain, offset=0.0, extra=None):
    """w_i = extra_i g_i / (d_i + b_i) where g_i (d_i + b_i) > 0, else 0 (float64).

    gain and offset are scalars or arrays of the data's shape; extra is None (1)
    or an array of that shape."""
    d = np.asarray(data, np.float64)
    g = np.broadcast_to(np.asarray(gain, np.float64), d.shape)
    b = np.broadcast_to(np.asarray(offset, np.float64), d.shape)
    e = np.ones_like(d) if extra is None else np.asarray(extra, np.float64)
    counts = g * (d + b)                                   # Eq. 18
    w = np.zeros_like(d)
    ok = counts > 0
    s2 = (d[ok] + b[ok]) / g[ok]                            # Eq. 21
    w[ok] = e[ok] / s2
    return w
