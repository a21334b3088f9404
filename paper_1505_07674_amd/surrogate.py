"""Learned surrogate of the log-likelihood that screens nested-sampling draws.

A multilayer perceptron 17 -> 256 -> 256 -> 256 -> 1 (SiLU), run and trained by
the library's bfloat16-MFMA kernels, is fitted to (theta, log L) pairs that the
exact likelihood produced during a nested-sampling run. It predicts
y = log(1 + L_ref - log L), the logarithm of the deficit from the best log L of
the training pairs (L_ref): the targets span the prior (deficit ~ 1e8) to the
posterior (deficit ~ 1-100) evenly, and a fixed error in y is a fixed
*relative* error of the deficit, so the network resolves a few nats near the
posterior where the screen needs them. The screen
discards a candidate when the predicted log L is below the current threshold by
more than a margin: three times the held-out root-mean-square error, in log L
units, of the held-out pairs whose log L is nearest the threshold. Every point
the sampler accepts is still evaluated exactly.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import torch

from . import binding
from .binding import MLP_NPARAM

IN, HID = 17, 256
LAYERS = (IN, HID, HID, HID, 1)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights for the SiLU layers, a small uniform head, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(4):
        n_in, n_out = LAYERS[i], LAYERS[i + 1]
        lim = math.sqrt(6.0 / n_in) if i < 3 else math.sqrt(1.0 / n_in)
        parts.append(rng.uniform(-lim, lim, size=n_out * n_in))
        parts.append(np.zeros(n_out))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == MLP_NPARAM
    return p


class Surrogate:
    def __init__(self, device: torch.device, seed: int = 0, free: Optional[np.ndarray] = None):
        self.device = device
        self.seed = seed
        self.free = None if free is None else np.asarray(free)
        self.params = torch.from_numpy(init_params(seed)).to(device)
        self.norm = None
        self.l_ref = 0.0
        self.margin_table = None      # (sorted held-out log L, running RMSE) for the margin
        self.history = []

    # -- inputs are points of the unit cube of the free parameters --------------
    def _x(self, u: np.ndarray) -> torch.Tensor:
        u = np.asarray(u, dtype=np.float32)
        if self.free is not None and u.shape[1] != IN:
            full = np.full((len(u), IN), 0.5, np.float32)
            full[:, self.free] = u
            u = full
        return torch.from_numpy(np.ascontiguousarray(u)).to(self.device)

    def fit(self, u: np.ndarray, logl: np.ndarray, epochs: int = 60, batch: int = 1024, lr: float = 2e-3,
            holdout: float = 0.1, seed: int = 0) -> dict:
        logl = np.asarray(logl, np.float64)
        ok = np.isfinite(logl)
        u, logl = np.asarray(u)[ok], logl[ok]
        self.l_ref = float(logl.max())
        y = np.log1p(self.l_ref - logl)
        rng = np.random.default_rng(seed)
        perm = rng.permutation(len(y))
        n_hold = max(int(holdout * len(y)), 1)
        hold, train = perm[:n_hold], perm[n_hold:]
        ym, ys = float(y[train].mean()), float(y[train].std() + 1e-12)
        norm = np.concatenate([np.full(IN, 0.5), np.full(IN, 2.0), [ym, ys]]).astype(np.float32)
        self.norm = torch.from_numpy(norm).to(self.device)
        X = self._x(u[train])
        Y = torch.from_numpy(y[train].astype(np.float32)).to(self.device)
        m = torch.zeros(MLP_NPARAM, device=self.device)
        v = torch.zeros(MLP_NPARAM, device=self.device)
        n = len(train)
        steps_per_epoch = max(n // batch, 1)
        total = epochs * steps_per_epoch
        step = 0
        loss = torch.empty(1, device=self.device)
        g = torch.Generator(device="cpu").manual_seed(seed)
        for ep in range(epochs):
            order = torch.randperm(n, generator=g).to(self.device)
            for b in range(steps_per_epoch):
                idx = order[b * batch:(b + 1) * batch]
                step += 1
                # cosine decay from lr to lr/100
                lr_t = lr * (0.01 + 0.99 * 0.5 * (1 + math.cos(math.pi * step / total)))
                binding.mlp_train_step(self.params, m, v, step, self.norm, X.index_select(0, idx).contiguous(),
                                       Y.index_select(0, idx).contiguous(), lr_t, loss=loss)
            if ep == epochs - 1 or ep % 10 == 0:
                self.history.append((ep, float(loss.cpu())))
        # held-out residuals in log L units, for the margin
        pred = self.predict(u[hold])
        res = pred - logl[hold]
        order = np.argsort(logl[hold])
        self.margin_table = (logl[hold][order], res[order])
        rmse_y = float(np.sqrt(np.mean((np.log1p(np.maximum(self.l_ref - pred, -0.999)) - y[hold]) ** 2)))
        return {"n_train": len(train), "n_holdout": n_hold, "final_loss": self.history[-1][1], "rmse_y": rmse_y,
                "l_ref": self.l_ref}

    def predict(self, u: np.ndarray) -> np.ndarray:
        """Predicted log L for unit-cube points."""
        if len(u) == 0:
            return np.zeros(0)
        y = binding.mlp_forward(self.params, self.norm, self._x(u)).double().cpu().numpy()
        return self.l_ref - np.expm1(y)

    def margin(self, lmin: float, k: int = 200, sigmas: float = 3.0, floor: float = 1.0) -> float:
        """sigmas x RMSE of the held-out residuals whose log L is nearest lmin."""
        ll, res = self.margin_table
        i = int(np.searchsorted(ll, lmin))
        lo, hi = max(0, i - k // 2), min(len(ll), i + k // 2)
        window = res[lo:hi] if hi > lo else res
        return max(sigmas * float(np.sqrt(np.mean(window ** 2))), floor)

    def save(self, path: str, fit: dict) -> None:
        """Weights, normalisation, reference log L, calibration table and fit summary (npz)."""
        import json
        np.savez(path, params=self.params.cpu().numpy(), norm=self.norm.cpu().numpy(), l_ref=np.asarray(self.l_ref),
                 cal_l=self.margin_table[0], cal_r=self.margin_table[1], fit=np.asarray(json.dumps(fit)))

    def load(self, path: str) -> dict:
        import json
        with np.load(path) as z:
            self.params = torch.from_numpy(z["params"]).to(self.device)
            self.norm = torch.from_numpy(z["norm"]).to(self.device)
            self.l_ref = float(z["l_ref"])
            self.margin_table = (z["cal_l"], z["cal_r"])
            return json.loads(str(z["fit"]))
