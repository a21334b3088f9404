"""Nested sampling for the forward-lensing likelihood.

The paper samples its posterior with nested sampling (Skilling 2004, 2006) via
the MultiNest library (Sec. 3.2), which needs only log P(d|xi) and returns the
posterior (Eq. 12) and the evidence (Eq. 13). This module is a plain
single-ellipsoid nested sampler that calls the batched GPU likelihood:

* live points are uniform in the unit cube, mapped to parameters by the prior
  transform (independent uniform priors);
* each iteration removes the k lowest-likelihood live points; the expected
  log-shrinkage of the prior volume for the j-th of them is -1/(n_live - j);
* replacements are drawn uniformly inside the bounding ellipsoid of the live
  points (enlarged by a volume factor, clipped to the cube) and accepted in draw
  order when their exact log L exceeds the threshold of the removed points;
* an optional screen (a trained surrogate) may discard candidates before the
  exact evaluation; every accepted point is evaluated exactly;
* the run stops when the live points can no longer change log Z by more than
  `dlogz`; the evidence error is sqrt(H / n_live) (Skilling 2006).
"""
from __future__ import annotations

import math
import pickle
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

LogLikeFn = Callable[[np.ndarray], np.ndarray]     # unit-cube points [m, d] -> float64 log L [m]


def _logaddexp(a, b):
    if a == -np.inf:
        return b
    if b == -np.inf:
        return a
    m = max(a, b)
    return m + math.log(math.exp(a - m) + math.exp(b - m))


class Ellipsoid:
    """Bounding ellipsoid of a point set, enlarged by a volume factor.

    ``sample_in_cube`` draws uniformly from the part of the ellipsoid inside the
    unit cube by whichever of two rejection schemes accepts more often: draws in
    the ellipsoid kept when inside the cube, or draws in the ellipsoid's bounding
    box (clipped to the cube) kept when inside the ellipsoid. Both give the same
    distribution; in many dimensions an ellipsoid that still spans the cube has a
    volume far larger than the cube, and one inside it a volume far smaller than
    its box, so neither scheme alone is efficient through a whole run.
    """

    def __init__(self, pts: np.ndarray, enlarge: float = 1.25):
        d = pts.shape[1]
        self.center = pts.mean(axis=0)
        cov = np.cov(pts, rowvar=False) + 1e-12 * np.eye(d)
        inv = np.linalg.inv(cov)
        delta = pts - self.center
        r2 = np.einsum("ij,jk,ik->i", delta, inv, delta).max()
        # scale so every point is inside, then enlarge the volume
        self.cov = cov * r2 * enlarge ** (2.0 / d)
        self.inv = np.linalg.inv(self.cov)
        self.chol = np.linalg.cholesky(self.cov)
        self.d = d
        half = np.sqrt(np.diag(self.cov))
        self.lo = np.clip(self.center - half, 0.0, 1.0)
        self.hi = np.clip(self.center + half, 0.0, 1.0)
        self._scheme = None

    def sample(self, rng: np.random.Generator, n: int) -> np.ndarray:
        z = rng.standard_normal((n, self.d))
        z /= np.linalg.norm(z, axis=1, keepdims=True)
        r = rng.random(n) ** (1.0 / self.d)
        return self.center + (z * r[:, None]) @ self.chol.T

    def contains(self, x: np.ndarray) -> np.ndarray:
        dlt = x - self.center
        return np.einsum("ij,jk,ik->i", dlt, self.inv, dlt) <= 1.0

    def _from_ellipsoid(self, rng, n):
        c = self.sample(rng, n)
        return c[np.all((c > 0.0) & (c < 1.0), axis=1)]

    def _from_box(self, rng, n):
        c = self.lo + rng.random((n, self.d)) * (self.hi - self.lo)
        return c[self.contains(c) & np.all(c > 0.0, axis=1)]

    def sample_in_cube(self, rng: np.random.Generator, n: int) -> np.ndarray:
        """Up to about n uniform draws from ellipsoid and cube (possibly fewer, never 0 twice in a row)."""
        if self._scheme is None:
            probe = 4096
            pa = len(self._from_ellipsoid(rng, probe)) / probe
            pb = len(self._from_box(rng, probe)) / probe
            self._scheme = (self._from_ellipsoid, max(pa, 1e-6)) if pa >= pb else (self._from_box, max(pb, 1e-6))
        fn, p = self._scheme
        m = int(min(max(n / p, n), 1 << 20))
        return fn(rng, m)


@dataclass
class Screen:
    """Pre-screen of candidates: predict(u) returns a log L estimate; a candidate
    is discarded when the estimate is below threshold - margin(threshold)."""
    predict: Callable[[np.ndarray], np.ndarray]
    margin: Callable[[float], float]
    max_skips: int = 2000           # consecutive discards before an exact fallback batch


@dataclass
class NSResult:
    logz: float
    logz_err: float
    samples: np.ndarray             # unit-cube points, dead then live
    logl: np.ndarray
    weights: np.ndarray             # posterior weights (sum to 1)
    n_exact: int                    # exact likelihood evaluations
    n_accepted: int                 # replacements accepted
    n_iter: int
    n_screened_out: int = 0
    n_audit: int = 0                # screened-out draws evaluated exactly to check the screen
    n_false_reject: int = 0         # of those, how many had log L above the threshold
    history: List[tuple] = field(default_factory=list)   # (n_exact, n_accepted) per iteration
    evaluated_u: Optional[np.ndarray] = None             # every exactly evaluated point
    evaluated_logl: Optional[np.ndarray] = None

    def posterior_moments(self, transform: Callable[[np.ndarray], np.ndarray]):
        x = transform(self.samples)
        mean = (self.weights[:, None] * x).sum(0)
        var = (self.weights[:, None] * (x - mean) ** 2).sum(0)
        return mean, np.sqrt(var)

    @property
    def renders_per_accepted(self) -> float:
        return self.n_exact / max(self.n_accepted, 1)


class NestedSampler:
    def __init__(self, loglike: LogLikeFn, ndim: int, n_live: int = 400, k_replace: int = 40,
                 enlarge: float = 1.25, dlogz: float = 0.5, seed: int = 0, max_iter: int = 100000,
                 candidates_per_call: int = 256, record: bool = False, audit: float = 0.0, audit_seed: int = 0):
        if not (1 <= k_replace < n_live):
            raise ValueError("need 1 <= k_replace < n_live")
        self.loglike = loglike
        self.ndim = ndim
        self.n_live = n_live
        self.k = k_replace
        self.enlarge = enlarge
        self.dlogz = dlogz
        self.rng = np.random.default_rng(seed)
        self.max_iter = max_iter
        self.cand = candidates_per_call
        self.record = record
        # audit: this fraction of screened-out draws is also evaluated exactly (not
        # accepted, not counted in n_exact) to measure false rejections
        self.audit = audit
        self.audit_rng = np.random.default_rng(audit_seed)
        self.state = None

    # -- checkpointing -------------------------------------------------------
    def checkpoint(self) -> bytes:
        return pickle.dumps({"state": self.state, "rng": self.rng.bit_generator.state})

    def restore(self, blob: bytes) -> None:
        d = pickle.loads(blob)
        self.state = d["state"]
        self.rng.bit_generator.state = d["rng"]

    # -- sampling ------------------------------------------------------------
    def _init_state(self):
        u = self.rng.random((self.n_live, self.ndim))
        logl = np.asarray(self.loglike(u), dtype=np.float64)
        self.state = {
            "live_u": u, "live_logl": logl, "dead_u": [], "dead_logl": [], "dead_logw": [],
            "logx": 0.0, "logz": -np.inf, "h": 0.0, "n_exact": self.n_live, "n_accepted": 0, "it": 0,
            "n_screened": 0, "history": [], "eval_u": [u] if self.record else [], "eval_l": [logl] if self.record else [],
            "rate": 0.5, "skips": 0, "audit_u": [], "n_audit": 0, "n_false_reject": 0,
        }

    def _draw(self, ell: Ellipsoid, m: int, lmin: float, screen: Optional[Screen]) -> np.ndarray:
        """The first m draws (in order) inside ellipsoid and cube that pass the screen."""
        st = self.state
        pool, have = [], 0
        while have < m:
            c = ell.sample_in_cube(self.rng, max(2 * m, 64))
            if len(c) == 0:
                continue
            if screen is not None and st["skips"] < screen.max_skips:
                keep = np.asarray(screen.predict(c)) >= lmin - screen.margin(lmin)
                # draws after the last kept one are not yet looked at: count discards up to it
                last = np.nonzero(keep)[0]
                looked = (last[-1] + 1) if len(last) else len(c)
                dropped = np.nonzero(~keep[:looked])[0]
                st["n_screened"] += len(dropped)
                if self.audit > 0 and len(dropped):
                    pick = dropped[self.audit_rng.random(len(dropped)) < self.audit]
                    if len(pick):
                        st["audit_u"].append(c[pick])
                st["skips"] = 0 if len(last) else st["skips"] + len(c)
                c = c[keep]
            else:
                st["skips"] = 0                    # exact fallback batch
            pool.append(c)
            have += len(c)
        return np.concatenate(pool)[:m]

    def _replace(self, lmin: float, n_new: int, screen: Optional[Screen]):
        st = self.state
        ell = Ellipsoid(st["live_u"], self.enlarge)
        new_u, new_l = [], []
        while len(new_u) < n_new:
            need = n_new - len(new_u)
            # size the exact batch from the running acceptance rate (about 10 % overshoot)
            m = min(self.cand * 16, int(math.ceil(1.1 * need / max(st["rate"], 1e-3))) + 1)
            c = self._draw(ell, m, lmin, screen)
            logl = np.asarray(self.loglike(c), dtype=np.float64)
            if st["audit_u"]:
                au = np.concatenate(st["audit_u"])
                st["audit_u"] = []
                al = np.asarray(self.loglike(au), dtype=np.float64)
                st["n_audit"] += len(au)
                st["n_false_reject"] += int(np.count_nonzero(al > lmin))
            st["n_exact"] += len(c)
            if self.record:
                st["eval_u"].append(c)
                st["eval_l"].append(logl)
            ok = np.nonzero(logl > lmin)[0]
            st["rate"] = 0.7 * st["rate"] + 0.3 * max(len(ok), 0.5) / len(c)
            for i in ok:                      # accept in draw order
                if len(new_u) < n_new:
                    new_u.append(c[i])
                    new_l.append(logl[i])
        st["n_accepted"] += n_new
        return np.array(new_u), np.array(new_l)

    def run(self, screen: Optional[Screen] = None, max_iter: Optional[int] = None,
            log: Optional[Callable[[str], None]] = None, log_every: int = 50,
            log_seconds: float = 20.0) -> NSResult:
        """Iterate until the stopping rule (or max_iter more iterations). ``log``
        receives a progress line every ``log_every`` iterations or ``log_seconds``
        seconds: iteration, L_min, log Z, exact evaluations, acceptance rate and
        screened-out draws."""
        if self.state is None:
            self._init_state()
        st = self.state
        n = self.n_live
        stop_at = st["it"] + (max_iter if max_iter is not None else self.max_iter)
        last_log = time.monotonic()
        while st["it"] < stop_at:
            order = np.argsort(st["live_logl"])
            worst = order[:self.k]
            lmin = st["live_logl"][worst[-1]]
            for j, idx in enumerate(worst):
                shrink = 1.0 / (n - j)
                logx_new = st["logx"] - shrink
                logw = st["live_logl"][idx] + st["logx"] + math.log(-math.expm1(-shrink))   # log(X - X')
                logz_new = _logaddexp(st["logz"], logw)
                # information H (Skilling 2006)
                if logz_new > -np.inf:
                    st["h"] = (math.exp(logw - logz_new) * st["live_logl"][idx]
                               + (math.exp(st["logz"] - logz_new) * (st["h"] + st["logz"]) if st["logz"] > -np.inf else 0.0)
                               - logz_new)
                st["logz"] = logz_new
                st["logx"] = logx_new
                st["dead_u"].append(st["live_u"][idx].copy())
                st["dead_logl"].append(st["live_logl"][idx])
                st["dead_logw"].append(logw)
            new_u, new_l = self._replace(lmin, self.k, screen)
            st["live_u"][worst] = new_u
            st["live_logl"][worst] = new_l
            st["it"] += 1
            st["history"].append((st["n_exact"], st["n_accepted"]))
            if log is not None and (st["it"] % log_every == 0 or time.monotonic() - last_log > log_seconds):
                last_log = time.monotonic()
                log(f"it {st['it']} lmin {lmin:.6g} logz {st['logz']:.6g} exact {st['n_exact']} "
                    f"accepted {st['n_accepted']} rate {st['rate']:.3g} screened {st['n_screened']}")
            # stop when the live points can add at most dlogz to log Z:
            # log(1 + L_max X / Z) < dlogz
            lmax = st["live_logl"].max()
            if self.dlogz > 0 and lmax + st["logx"] - st["logz"] < math.log(math.expm1(self.dlogz)):
                break
        return self._result()

    def _result(self) -> NSResult:
        st = self.state
        n = self.n_live
        live_logw = st["live_logl"] + st["logx"] - math.log(n)
        logw = np.concatenate([np.array(st["dead_logw"]), live_logw])
        logz = st["logz"]
        for lw in live_logw:
            logz = _logaddexp(logz, lw)
        w = np.exp(logw - logz)
        w /= w.sum()
        samples = np.concatenate([np.array(st["dead_u"]).reshape(-1, self.ndim), st["live_u"]])
        logl = np.concatenate([np.array(st["dead_logl"]), st["live_logl"]])
        h = max(st["h"], 0.0)
        res = NSResult(logz=logz, logz_err=math.sqrt(h / n), samples=samples, logl=logl, weights=w,
                       n_exact=st["n_exact"], n_accepted=st["n_accepted"], n_iter=st["it"],
                       n_screened_out=st["n_screened"], history=list(st["history"]),
                       n_audit=st["n_audit"], n_false_reject=st["n_false_reject"])
        if self.record and st["eval_u"]:
            res.evaluated_u = np.concatenate(st["eval_u"])
            res.evaluated_logl = np.concatenate(st["eval_l"])
        return res
