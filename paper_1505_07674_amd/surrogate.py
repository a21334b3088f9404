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
    """Network, target transform and input feature map.

    Inputs: the sampler's unit-cube coordinates of the free parameters. The
    host maps them to the network input by an affine feature map x = P^T (u - mu)
    (fixed parameters enter as 0): for the global fit mu = 1/2, P = 2 I (the cube
    onto [-1, 1]); a local refit whitens by the principal axes of its pairs, so
    that a narrow, strongly correlated posterior becomes a unit-scale problem.
    The kernels' own input normalisation is the identity."""

    def __init__(self, device: torch.device, seed: int = 0, free: Optional[np.ndarray] = None):
        self.device = device
        self.seed = seed
        self.free = np.arange(IN) if free is None else np.asarray(free)
        nf = len(self.free)
        self.mu = np.full(nf, 0.5)
        self.P = 2.0 * np.eye(nf)
        self.params = torch.from_numpy(init_params(seed)).to(device)
        self.norm = None
        self.l_ref = 0.0
        self.margin_table = None      # (sorted held-out log L, residual) for the margin
        self.history = []

    def _x(self, u: np.ndarray) -> torch.Tensor:
        u = np.asarray(u, dtype=np.float64)
        if u.shape[1] == IN and len(self.free) != IN:
            u = u[:, self.free]
        x = np.zeros((len(u), IN), np.float32)
        x[:, self.free] = (u - self.mu) @ self.P
        return torch.from_numpy(x).to(self.device)

    def _set_norm(self, ym: float, ys: float) -> None:
        norm = np.concatenate([np.zeros(IN), np.ones(IN), [ym, ys]]).astype(np.float32)
        self.norm = torch.from_numpy(norm).to(self.device)

    def _train(self, X: torch.Tensor, Y: torch.Tensor, steps: int, batch: int, lr: float, seed: int) -> float:
        """Adam on (X, Y) for `steps` mini-batches, cosine decay from lr to lr/100."""
        n = X.shape[0]
        batch = min(batch, n)
        m = torch.zeros(MLP_NPARAM, device=self.device)
        v = torch.zeros(MLP_NPARAM, device=self.device)
        loss = torch.empty(1, device=self.device)
        g = torch.Generator(device="cpu").manual_seed(seed)
        order = torch.randperm(n, generator=g).to(self.device)
        pos = 0
        for step in range(1, steps + 1):
            if pos + batch > n:
                order = torch.randperm(n, generator=g).to(self.device)
                pos = 0
            idx = order[pos:pos + batch]
            pos += batch
            lr_t = lr * (0.01 + 0.99 * 0.5 * (1 + math.cos(math.pi * step / steps)))
            binding.mlp_train_step(self.params, m, v, step, self.norm, X.index_select(0, idx).contiguous(),
                                   Y.index_select(0, idx).contiguous(), lr_t, loss=loss)
        return float(loss.cpu())

    def _calibrate(self, u: np.ndarray, logl: np.ndarray, y: np.ndarray) -> float:
        pred = self.predict(u)
        order = np.argsort(logl)
        self.margin_table = (logl[order], (pred - logl)[order])
        return float(np.sqrt(np.mean((np.log1p(np.maximum(self.l_ref - pred, -0.999)) - y) ** 2)))

    def fit(self, u: np.ndarray, logl: np.ndarray, epochs: int = 60, batch: int = 1024, lr: float = 2e-3,
            holdout: float = 0.1, seed: int = 0) -> dict:
        """Global fit on a run's pairs; inputs are the unit cube mapped to [-1, 1]."""
        logl = np.asarray(logl, np.float64)
        ok = np.isfinite(logl)
        u, logl = np.asarray(u)[ok], logl[ok]
        self.l_ref = float(logl.max())
        y = np.log1p(self.l_ref - logl)
        rng = np.random.default_rng(seed)
        perm = rng.permutation(len(y))
        n_hold = max(int(holdout * len(y)), 1)
        hold, train = perm[:n_hold], perm[n_hold:]
        self.mu = np.full(len(self.free), 0.5)
        self.P = 2.0 * np.eye(len(self.free))
        self._set_norm(float(y[train].mean()), float(y[train].std() + 1e-12))
        X = self._x(u[train])
        Y = torch.from_numpy(y[train].astype(np.float32)).to(self.device)
        steps = epochs * max(len(train) // batch, 1)
        final = self._train(X, Y, steps, batch, lr, seed)
        self.history.append(("fit", final))
        rmse_y = self._calibrate(u[hold], logl[hold], y[hold])
        return {"n_train": len(train), "n_holdout": n_hold, "final_loss": final, "rmse_y": rmse_y,
                "l_ref": self.l_ref}

    def _remap(self, mu_new: np.ndarray, P_new: np.ndarray) -> None:
        """Change the feature map to x = P_new^T (u - mu_new) without changing the
        network's function of u: W1_f x_old + b1 = W1_f P_old^T (u - mu_old) + b1, so
        W1_f' = W1_f P_old^T P_new^{-T} and b1' = b1 + W1_f P_old^T (mu_new - mu_old)."""
        p = self.params.double().cpu().numpy()
        W1 = p[:HID * IN].reshape(HID, IN)
        Wf = W1[:, self.free]
        M = self.P.T @ np.linalg.inv(P_new).T
        b1 = p[HID * IN:HID * IN + HID] + Wf @ (self.P.T @ (mu_new - self.mu))
        W1[:, self.free] = Wf @ M
        p[:HID * IN] = W1.reshape(-1)
        p[HID * IN:HID * IN + HID] = b1
        self.params = torch.from_numpy(p.astype(np.float32)).to(self.device)
        self.mu, self.P = np.asarray(mu_new, np.float64), np.asarray(P_new, np.float64)

    def refit(self, u: np.ndarray, logl: np.ndarray, steps: int = 300, batch: int = 1024, lr: float = 1e-3,
              holdout: float = 0.1, seed: int = 0) -> dict:
        """Local refit on the pairs of the current contour region. The feature map
        becomes the whitening of these pairs (scaled to about [-1, 1]); the first
        layer is transformed so that the network computes the same function of
        theta as before, and training continues from there. L_ref becomes the
        best log L of the pairs; the held-out tenth recalibrates the margin."""
        logl = np.asarray(logl, np.float64)
        ok = np.isfinite(logl)
        u, logl = np.asarray(u, np.float64)[ok], logl[ok]
        if u.shape[1] == IN and len(self.free) != IN:
            u = u[:, self.free]
        mu_new = u.mean(axis=0)
        ev, V = np.linalg.eigh(np.cov(u, rowvar=False) + 1e-30 * np.eye(u.shape[1]))
        P_new = V / (2.0 * np.sqrt(np.maximum(ev, 1e-300)))
        self._remap(mu_new, P_new)
        self.l_ref = float(logl.max()) + 1.0
        y = np.log1p(self.l_ref - logl)
        rng = np.random.default_rng(seed)
        perm = rng.permutation(len(y))
        n_hold = max(int(holdout * len(y)), 1)
        hold, train = perm[:n_hold], perm[n_hold:]
        self._set_norm(float(y[train].mean()), float(y[train].std() + 1e-12))
        X = self._x(u[train])
        Y = torch.from_numpy(y[train].astype(np.float32)).to(self.device)
        final = self._train(X, Y, steps, batch, lr, seed)
        self.history.append(("refit", final))
        rmse_y = self._calibrate(u[hold], logl[hold], y[hold])
        return {"n_train": len(train), "final_loss": final, "rmse_y": rmse_y, "l_ref": self.l_ref}

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

    def snapshot(self) -> dict:
        """An in-memory copy of the trained state (weights, maps, calibration)."""
        return {"params": self.params.clone(), "norm": None if self.norm is None else self.norm.clone(),
                "l_ref": self.l_ref, "mu": self.mu.copy(), "P": self.P.copy(),
                "margin_table": None if self.margin_table is None else tuple(a.copy() for a in self.margin_table),
                "history": list(self.history)}

    def restore(self, snap: dict) -> None:
        """Back to a snapshot (so that several screened runs start from the same network)."""
        self.params = snap["params"].clone()
        self.norm = None if snap["norm"] is None else snap["norm"].clone()
        self.l_ref = snap["l_ref"]
        self.mu, self.P = snap["mu"].copy(), snap["P"].copy()
        self.margin_table = None if snap["margin_table"] is None else tuple(a.copy() for a in snap["margin_table"])
        self.history = list(snap["history"])

    def save(self, path: str, fit: dict) -> None:
        """Weights, normalisation, reference log L, calibration table and fit summary (npz)."""
        import json
        np.savez(path, params=self.params.cpu().numpy(), norm=self.norm.cpu().numpy(), l_ref=np.asarray(self.l_ref),
                 mu=self.mu, P=self.P, cal_l=self.margin_table[0], cal_r=self.margin_table[1],
                 fit=np.asarray(json.dumps(fit)))

    def load(self, path: str) -> dict:
        import json
        with np.load(path) as z:
            self.params = torch.from_numpy(z["params"]).to(self.device)
            self.norm = torch.from_numpy(z["norm"]).to(self.device)
            self.l_ref = float(z["l_ref"])
            self.mu, self.P = z["mu"], z["P"]
            self.margin_table = (z["cal_l"], z["cal_r"])
            return json.loads(str(z["fit"]))
