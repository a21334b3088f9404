"""Nested sampling for the forward-lensing likelihood.

The paper samples its posterior with nested sampling (Skilling 2004, 2006) via
the MultiNest library (Sec. 3.2), which needs only log P(d|xi) and returns the
posterior (Eq. 12) and the evidence (Eq. 13). This module is a nested sampler
that calls the batched GPU likelihood:

* live points are uniform in the unit cube, mapped to parameters by the prior
  transform (independent uniform priors);
* each iteration removes the k lowest-likelihood live points; the expected
  log-shrinkage of the prior volume for the j-th of them is -1/(n_live - j);
* replacements are drawn uniformly inside the bounding ellipsoids of the live
  points (a union found by recursive 2-means splits, as MultiNest does, each
  enlarged by a volume factor, clipped to the cube) and accepted in draw order
  when their exact log L exceeds the threshold of the removed points, or come
  from slice-sampling chains (Neal 2003) started at surviving live points, as
  PolyChord does, whichever costs fewer exact evaluations per replacement;
* an optional screen (a trained surrogate) may discard candidates before the
  exact evaluation; every accepted point, and every point a slice chain moves
  to, is evaluated exactly;
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


def _two_means(pts: np.ndarray, rng: np.random.Generator, iters: int = 20) -> np.ndarray:
    """Labels (0/1) of a 2-means clustering, started from two far-apart points."""
    a = pts[rng.integers(len(pts))]
    c0 = pts[np.argmax(np.sum((pts - a) ** 2, axis=1))]
    c1 = pts[np.argmax(np.sum((pts - c0) ** 2, axis=1))]
    lab = np.zeros(len(pts), dtype=int)
    for _ in range(iters):
        new = (np.sum((pts - c1) ** 2, axis=1) < np.sum((pts - c0) ** 2, axis=1)).astype(int)
        if np.array_equal(new, lab) and _ > 0:
            break
        lab = new
        if lab.all() or not lab.any():
            break
        c0, c1 = pts[lab == 0].mean(axis=0), pts[lab == 1].mean(axis=0)
    return lab


def _log_volume(cov: np.ndarray) -> float:
    return 0.5 * np.linalg.slogdet(cov)[1]


class MultiEllipsoid:
    """Union of ellipsoids bounding the live points (Feroz & Hobson 2008): the
    set is split recursively by 2-means while the two children's bounding
    ellipsoids together take less than half the parent's volume; each ellipsoid
    is enlarged by enlarge * sqrt(n_live / n_cluster) in volume (at most 4x).
    Draws are uniform over the union inside the cube: pick an ellipsoid with
    probability proportional to its volume, draw in it, keep the draw with
    probability 1 / (number of ellipsoids containing it). A single ellipsoid
    uses Ellipsoid.sample_in_cube."""

    def __init__(self, pts: np.ndarray, enlarge: float = 1.25, rng: Optional[np.random.Generator] = None,
                 max_ellipsoids: int = 16):
        self.d = pts.shape[1]
        self.n = len(pts)
        self.enlarge = enlarge
        rng = rng if rng is not None else np.random.default_rng(0)
        self.ells: List[Ellipsoid] = []
        stack = [pts]
        while stack:
            p = stack.pop()
            e = self._fit(p)
            if len(p) >= 2 * (self.d + 1) and len(self.ells) + len(stack) + 2 <= max_ellipsoids:
                lab = _two_means(p, rng)
                p0, p1 = p[lab == 0], p[lab == 1]
                if len(p0) > self.d + 1 and len(p1) > self.d + 1:
                    e0, e1 = self._fit(p0), self._fit(p1)
                    lv = _log_volume(e.cov)
                    if np.logaddexp(_log_volume(e0.cov), _log_volume(e1.cov)) < lv + math.log(0.5):
                        stack.extend([p0, p1])
                        continue
            self.ells.append(e)
        lv = np.array([_log_volume(e.cov) for e in self.ells])
        w = np.exp(lv - lv.max())
        self.prob = w / w.sum()

    def _fit(self, p: np.ndarray) -> Ellipsoid:
        f = min(self.enlarge * math.sqrt(self.n / len(p)), 4.0)
        return Ellipsoid(p, f)

    def sample_in_cube(self, rng: np.random.Generator, n: int) -> np.ndarray:
        if len(self.ells) == 1:
            return self.ells[0].sample_in_cube(rng, n)
        counts = rng.multinomial(n, self.prob)
        parts = [e.sample(rng, k) for e, k in zip(self.ells, counts) if k > 0]
        c = np.concatenate(parts)
        c = c[np.all((c > 0.0) & (c < 1.0), axis=1)]
        if len(c) == 0:
            return c
        inside = np.sum([e.contains(c) for e in self.ells], axis=0)
        keep = rng.random(len(c)) * np.maximum(inside, 1) < 1.0
        c = c[keep]
        return c[rng.permutation(len(c))]


@dataclass
class Screen:
    """Pre-screen of candidates: predict(u) returns a log L estimate; a candidate
    is discarded when the estimate is below threshold - margin(threshold).

    A slice chain uses the screen in two ways. While it steps its interval out,
    a proposal whose estimate clears threshold + margin_in(threshold)
    (margin(threshold) when the screen has no margin_in) counts as inside
    without an exact render: the interval is then built from a fixed,
    deterministic set, which leaves slice sampling's uniform target intact. A
    chain only ever moves to a proposal rendered exactly above the threshold;
    there the screen may only discard. So the screen's false discards are the
    one way it can bias a run, in slice and rejection mode alike: both then
    sample the contour minus the discarded region."""
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
    n_trusted: int = 0              # step-out proposals the screen classified as inside (no exact render)
    n_false_accept: int = 0         # audited trusted proposals whose exact log L was below the threshold
    n_fallback: int = 0             # slice chains rerun without the screen
    history: List[tuple] = field(default_factory=list)   # (n_exact, n_accepted) per iteration
    evaluated_u: Optional[np.ndarray] = None             # every exactly evaluated point
    evaluated_logl: Optional[np.ndarray] = None

    def posterior_moments(self, transform: Callable[[np.ndarray], np.ndarray]):
        x = transform(self.samples)
        mean = (self.weights[:, None] * x).sum(0)
        var = (self.weights[:, None] * (x - mean) ** 2).sum(0)
        return mean, np.sqrt(var)

    converged: bool = False         # the stopping rule fired (else max_iter ended the run)

    @property
    def renders_per_accepted(self) -> float:
        return self.n_exact / max(self.n_accepted, 1)


class NestedSampler:
    def __init__(self, loglike: LogLikeFn, ndim: int, n_live: int = 400, k_replace: int = 40,
                 enlarge: float = 1.25, dlogz: float = 0.5, seed: int = 0, max_iter: int = 100000,
                 candidates_per_call: int = 256, record: bool = False, audit: float = 0.0, audit_seed: int = 0,
                 multi: bool = True, record_per_iter: Optional[int] = None,
                 audit_loglike: Optional[LogLikeFn] = None, method: str = "auto", n_steps: Optional[int] = None,
                 slice_switch: Optional[float] = None, probe_every: int = 20):
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
        self.audit_loglike = audit_loglike if audit_loglike is not None else loglike
        # record: keep exact (u, log L) pairs, at most record_per_iter per iteration
        # (a uniform subset, drawn with its own generator)
        self.record_per_iter = record_per_iter
        self.record_rng = np.random.default_rng(audit_seed + 2)
        # method: "rejection" (draws inside bounding ellipsoids), "slice" (slice
        # sampling chains), or "auto": per iteration the one with the lower
        # measured exact renders per replacement (see _replace_auto)
        if method not in ("auto", "rejection", "slice"):
            raise ValueError("method must be auto, rejection or slice")
        self.method = method
        self.n_steps = n_steps if n_steps is not None else ndim
        # before any slice iteration has been measured, rejection is tried with a
        # budget of twice this guess of the slice cost (renders per replacement)
        self.slice_cost_guess = 1.0 / slice_switch if slice_switch is not None else 5.0 * self.n_steps
        self.probe_every = probe_every
        # multi: bound the live points by a union of ellipsoids (else one ellipsoid)
        self.multi = multi
        self.split_rng = np.random.default_rng(seed + 1)
        self.state = None

    # -- checkpointing -------------------------------------------------------
    def checkpoint(self) -> bytes:
        return pickle.dumps({"state": self.state, "rng": self.rng.bit_generator.state,
                             "split_rng": self.split_rng.bit_generator.state,
                             "audit_rng": self.audit_rng.bit_generator.state,
                             "record_rng": self.record_rng.bit_generator.state})

    def restore(self, blob: bytes) -> None:
        """Resume from a checkpoint() blob this program wrote (pickle: trusted input only)."""
        d = pickle.loads(blob)
        self.state = d["state"]
        self.rng.bit_generator.state = d["rng"]
        self.split_rng.bit_generator.state = d["split_rng"]
        self.audit_rng.bit_generator.state = d["audit_rng"]
        self.record_rng.bit_generator.state = d["record_rng"]

    # -- sampling ------------------------------------------------------------
    def _init_state(self):
        u = self.rng.random((self.n_live, self.ndim))
        logl = np.asarray(self.loglike(u), dtype=np.float64)
        self.state = {
            "live_u": u, "live_logl": logl, "dead_u": [], "dead_logl": [], "dead_logw": [],
            "logx": 0.0, "logz": -np.inf, "h": 0.0, "n_exact": self.n_live, "n_accepted": 0, "it": 0,
            "n_screened": 0, "history": [], "eval_u": [u.astype(np.float32)] if self.record else [],
            "eval_l": [logl.copy()] if self.record else [],
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
                st["drawn_it"] += looked
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
                st["drawn_it"] += min(len(c), m - have)
            pool.append(c)
            have += len(c)
        return np.concatenate(pool)[:m]

    def _exact(self, c: np.ndarray) -> np.ndarray:
        """Exact log L of the points c (counted, and recorded when asked)."""
        st = self.state
        logl = np.asarray(self.loglike(c), dtype=np.float64)
        st["n_exact"] += len(c)
        if self.record:
            take = np.arange(len(c))
            if self.record_per_iter is not None:
                room = self.record_per_iter - st.get("rec_it", 0)
                take = take[self.record_rng.random(len(c)) < min(1.0, max(room, 0) / max(len(c), 1))]
                st["rec_it"] = st.get("rec_it", 0) + len(take)
            st["eval_u"].append(c[take].astype(np.float32))
            st["eval_l"].append(logl[take])
        return logl

    def _audit(self, lmin: float) -> None:
        st = self.state
        if st["audit_u"]:
            au = np.concatenate(st["audit_u"])
            st["audit_u"] = []
            al = np.asarray(self.audit_loglike(au), dtype=np.float64)
            st["n_audit"] += len(au)
            st["n_false_reject"] += int(np.count_nonzero(al > lmin))
        if st.get("audit_in"):
            au = np.concatenate(st["audit_in"])
            st["audit_in"] = []
            al = np.asarray(self.audit_loglike(au), dtype=np.float64)
            st["n_audit"] += len(au)
            st["n_false_accept"] = st.get("n_false_accept", 0) + int(np.count_nonzero(al <= lmin))

    def _replace(self, lmin: float, n_new: int, screen: Optional[Screen]):
        st = self.state
        st["rec_it"] = 0
        st["drawn_it"] = 0
        if self.method == "slice":
            out = self._replace_slice(lmin, n_new, screen)
        elif self.method == "rejection":
            out = self._replace_rejection(lmin, n_new, screen)
        else:
            out = self._replace_auto(lmin, n_new, screen)
        st["n_accepted"] += n_new
        return out

    def _replace_auto(self, lmin: float, n_new: int, screen: Optional[Screen]):
        """Rejection or slice replacements, whichever has cost fewer exact renders
        per accepted point lately (running averages); every probe_every
        iterations the other one is tried, rejection with a render budget of
        twice the slice cost (the shortfall is filled by slice)."""
        st = self.state
        c_rej, c_sl = st.get("cost_rej"), st.get("cost_slice")
        use_rej = c_sl is None or (c_rej is not None and c_rej <= c_sl)
        since = st["it"] - st.get("last_probe", -10 ** 9)
        if since >= self.probe_every and c_rej is not None and c_sl is not None:
            use_rej = not use_rej
            st["last_probe"] = st["it"]
        n0 = st["n_exact"]
        if use_rej:
            budget = None if c_sl is None else int(2.0 * c_sl * n_new) + 1
            if c_sl is None and c_rej is not None and c_rej > self.slice_cost_guess:
                budget = int(2.0 * self.slice_cost_guess * n_new) + 1
            u, l = self._replace_rejection(lmin, n_new, screen, budget=budget)
            got = len(u)
            if got:
                st["cost_rej"] = self._ema(c_rej, (st["n_exact"] - n0) / got)
            else:
                st["cost_rej"] = self._ema(c_rej, float(st["n_exact"] - n0 + 1))
            if got < n_new:
                n1 = st["n_exact"]
                us, ls = self._replace_slice(lmin, n_new - got, screen)
                st["cost_slice"] = self._ema(c_sl, (st["n_exact"] - n1) / (n_new - got))
                u = us if got == 0 else np.concatenate([u, us])
                l = ls if got == 0 else np.concatenate([l, ls])
            return u, l
        u, l = self._replace_slice(lmin, n_new, screen)
        st["cost_slice"] = self._ema(c_sl, (st["n_exact"] - n0) / n_new)
        return u, l

    @staticmethod
    def _ema(old: Optional[float], new: float) -> float:
        return new if old is None else 0.7 * old + 0.3 * new

    def _replace_rejection(self, lmin: float, n_new: int, screen: Optional[Screen], budget: Optional[int] = None):
        """Up to n_new replacements drawn in the bound; with a budget, stops once
        that many exact renders were spent (possibly returning fewer)."""
        st = self.state
        ell = (MultiEllipsoid(st["live_u"], self.enlarge, self.split_rng) if self.multi
               else Ellipsoid(st["live_u"], self.enlarge))
        new_u, new_l = [], []
        n0 = st["n_exact"]
        while len(new_u) < n_new:
            if budget is not None and st["n_exact"] - n0 >= budget:
                break
            need = n_new - len(new_u)
            # size the exact batch from the running acceptance rate (about 10 % overshoot)
            m = min(self.cand * 16, int(math.ceil(1.1 * need / max(st["rate"], 1e-3))) + 1)
            c = self._draw(ell, m, lmin, screen)
            logl = self._exact(c)
            self._audit(lmin)
            ok = np.nonzero(logl > lmin)[0]
            st["rate"] = 0.7 * st["rate"] + 0.3 * max(len(ok), 0.5) / len(c)
            for i in ok:                      # accept in draw order
                if len(new_u) < n_new:
                    new_u.append(c[i])
                    new_l.append(logl[i])
        return np.array(new_u).reshape(-1, self.ndim), np.array(new_l)

    def _classify(self, c: np.ndarray, lmin: float, screen: Optional[Screen], trust_in: np.ndarray):
        """Inside-the-contour flags for proposals c (points outside the cube are
        outside): by the screen where its prediction falls below L_min by the
        margin, or (where trust_in is set) clears it by the inside margin; exactly
        otherwise. Returns (inside, exact log L or nan)."""
        st = self.state
        inside = np.zeros(len(c), dtype=bool)
        logl = np.full(len(c), np.nan)
        cube = np.all((c > 0.0) & (c < 1.0), axis=1)
        todo = np.nonzero(cube)[0]
        if screen is not None and len(todo) and st["skips"] < screen.max_skips:
            pred = np.asarray(screen.predict(c[todo]))
            dm = screen.margin(lmin)
            dm_in = screen.margin_in(lmin) if hasattr(screen, "margin_in") else dm
            sure_in, sure_out = (pred > lmin + dm_in) & trust_in[todo], pred < lmin - dm
            inside[todo[sure_in]] = True
            st["n_screened"] += int(sure_out.sum())
            st["n_trusted"] = st.get("n_trusted", 0) + int(sure_in.sum())
            if self.audit > 0:
                pick_out = todo[sure_out][self.audit_rng.random(int(sure_out.sum())) < self.audit]
                pick_in = todo[sure_in][self.audit_rng.random(int(sure_in.sum())) < self.audit]
                if len(pick_out):
                    st["audit_u"].append(c[pick_out])
                if len(pick_in):
                    st.setdefault("audit_in", []).append(c[pick_in])
            todo = todo[~(sure_in | sure_out)]
        if len(todo):
            logl[todo] = self._exact(c[todo])
            inside[todo] = logl[todo] > lmin
        return inside, logl

    def _replace_slice(self, lmin: float, n_new: int, screen: Optional[Screen]):
        """n_new replacements by slice sampling (Neal 2003) inside the contour,
        one chain per replacement from a random surviving live point, along random
        directions whitened by the live points' covariance (as PolyChord does),
        n_steps slices per chain, all chains advanced in lock-step so that every
        round is one batched evaluation. With a screen, step-out proposals whose
        predicted log L clears the threshold by the margin count as inside without
        an exact render, and any proposal predicted below it by the margin counts
        as outside; a chain moves only to a proposal whose exact log L exceeds the
        threshold, so every point of a chain is exactly inside. A chain whose slice
        shrinks to nothing is rerun without the screen."""
        st = self.state
        live = st["live_u"]
        keep = np.nonzero(st["live_logl"] > lmin)[0]
        if len(keep) == 0:
            keep = np.arange(len(live))
        cov = np.cov(live[keep], rowvar=False) + 1e-12 * np.eye(self.ndim)
        chol = np.linalg.cholesky(cov)
        B = n_new
        start = keep[self.rng.integers(len(keep), size=B)]
        x = live[start].copy()
        xl = st["live_logl"][start].copy()          # exact log L of x (nan when only screened)
        out_u, out_l = np.zeros((B, self.ndim)), np.zeros(B)
        pending = np.arange(B)
        use_screen = screen
        for attempt in range(3):
            steps = np.zeros(B, dtype=int)
            def new_dir(idx):
                e = self.rng.standard_normal((len(idx), self.ndim))
                e /= np.linalg.norm(e, axis=1, keepdims=True)
                return e @ chol.T
            v = np.zeros((B, self.ndim))
            v[pending] = new_dir(pending)
            lo = np.zeros(B)
            lo[pending] = -self.rng.random(len(pending))
            hi = lo + 1.0
            phase = np.full(B, 3)                    # 0 step out low, 1 step out high, 2 shrink, 3 done
            phase[pending] = 0
            nout = np.zeros(B, dtype=int)
            nshrink = np.zeros(B, dtype=int)
            failed = np.zeros(B, dtype=bool)
            while True:
                act = np.nonzero(phase < 3)[0]
                if len(act) == 0:
                    break
                t = np.where(phase[act] == 0, lo[act], np.where(phase[act] == 1, hi[act], 0.0))
                sh = phase[act] == 2
                t[sh] = lo[act][sh] + self.rng.random(int(sh.sum())) * (hi[act][sh] - lo[act][sh])
                prop = x[act] + t[:, None] * v[act]
                # a move (shrinkage phase) needs the exact log L; stepping out may trust the screen
                inside, pl = self._classify(prop, lmin, use_screen, trust_in=~sh)
                for j, i in enumerate(act):
                    if phase[i] == 0:
                        if inside[j] and nout[i] < 20:
                            lo[i] -= 1.0
                            nout[i] += 1
                        else:
                            phase[i], nout[i] = 1, 0
                    elif phase[i] == 1:
                        if inside[j] and nout[i] < 20:
                            hi[i] += 1.0
                            nout[i] += 1
                        else:
                            phase[i] = 2
                    else:
                        if inside[j]:
                            x[i], xl[i] = prop[j], pl[j]
                            steps[i] += 1
                            if steps[i] >= self.n_steps:
                                phase[i] = 3
                            else:
                                v[i] = new_dir(np.array([i]))[0]
                                lo[i] = -self.rng.random()
                                hi[i] = lo[i] + 1.0
                                phase[i], nout[i], nshrink[i] = 0, 0, 0
                        else:
                            if t[j] < 0.0:
                                lo[i] = t[j]
                            else:
                                hi[i] = t[j]
                            nshrink[i] += 1
                            if nshrink[i] > 60:      # the neighbourhood of x reads as outside
                                failed[i], phase[i] = True, 3
            # every replacement carries an exact log L above the threshold
            done = pending[~failed[pending]]
            ok = done[xl[done] > lmin]
            out_u[ok], out_l[ok] = x[ok], xl[ok]
            self._audit(lmin)
            pending = np.setdiff1d(pending, ok)
            if len(pending) == 0:
                break
            # fallback: rerun the failed chains from live points without the screen
            st["n_fallback"] = st.get("n_fallback", 0) + len(pending)
            start = keep[self.rng.integers(len(keep), size=len(pending))]
            x[pending], xl[pending] = live[start], st["live_logl"][start]
            use_screen = None
        if len(pending):
            # last resort: bounded rejection draws, exact
            u, l = self._replace_rejection(lmin, len(pending), None)
            out_u[pending], out_l[pending] = u, l
        return out_u, out_l

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
        while st["it"] < stop_at and not st.get("done", False):
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
            if screen is not None and hasattr(screen, "begin_iteration"):
                screen.begin_iteration(lmin, st["it"])
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
                st["done"] = True
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
                       n_audit=st["n_audit"], n_false_reject=st["n_false_reject"],
                       n_trusted=st.get("n_trusted", 0), n_false_accept=st.get("n_false_accept", 0),
                       n_fallback=st.get("n_fallback", 0),
                       converged=bool(st.get("done", False)))
        if self.record and st["eval_u"]:
            res.evaluated_u = np.concatenate(st["eval_u"])
            res.evaluated_logl = np.concatenate(st["eval_l"])
        return res
