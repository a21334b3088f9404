"""Nested sampling with and without the learned screen, on the GPU likelihood.

``GpuLogLike`` turns unit-cube points of the free parameters into float64 log L
through the batched library path (one graph launch per call of at most
``max_batch`` points; longer calls are split). It pads every call up to a
power-of-two bucket so that the library's cached launch plans are reused
instead of rebuilt for each new batch size; padding rows are copies of the
first point and are not counted as evaluations.

``SurrogateScreen`` wraps a trained ``Surrogate`` as the sampler's screen. Its
margin starts from the held-out residuals and is recalibrated as the run goes:
every candidate that passes the screen is evaluated exactly, and its residual
(prediction minus exact log L) joins the calibration set. The margin at a
threshold L_min is ``sigmas`` times the root-mean-square residual of the
calibration pairs whose exact log L is nearest L_min. The run's own residuals
are kept for the most recent ``keep`` evaluations: the threshold only rises, so
older pairs lie below it.

``ScreenExperiment`` (and ``compare_runs``, all of it in one call) is the
end-to-end experiment: a plain run that records every exact (theta, log L)
pair, a second plain run with another seed (the null spread of the sampler
itself), the surrogate trained on the first run's pairs, and a screened run; it
reports exact renders per accepted point and the posterior mean shifts in units
of the plain posterior standard deviation.
"""
from __future__ import annotations

import math
import time
from typing import Dict, Optional

import numpy as np
import torch

from . import binding
from .mocks import Observation, SystemSpec
from .sampler import NestedSampler, NSResult, Screen
from .surrogate import Surrogate


class GpuLogLike:
    def __init__(self, spec: SystemSpec, obs: Observation, device: torch.device, min_bucket: int = 64,
                 ctx: Optional[binding.Context] = None, max_batch: int = 16384):
        self.spec = spec
        self.device = device
        self.free = spec.prior.free
        self.ctx = ctx or binding.Context(device.index or 0)
        self.system = binding.System(torch.from_numpy(spec.psf).to(device), torch.from_numpy(obs.data).to(device),
                                     torch.from_numpy(obs.weight).to(device), pixscale=spec.pixscale,
                                     nsub=spec.nsub, center=(spec.center_x, spec.center_y))
        self.min_bucket, self.max_batch = min_bucket, max_batch
        self.buffers: Dict[int, tuple] = {}
        self.n_calls = 0
        self.n_points = 0
        self.gpu_s = 0.0

    def theta(self, u: np.ndarray) -> np.ndarray:
        lo, hi = self.spec.prior.low, self.spec.prior.high
        full = np.tile(lo, (len(u), 1))
        full[:, self.free] = lo[self.free] + np.asarray(u) * (hi - lo)[self.free]
        return full.astype(np.float32)

    def __call__(self, u: np.ndarray) -> np.ndarray:
        u = np.atleast_2d(np.asarray(u))
        n = len(u)
        if n == 0:
            return np.zeros(0)
        if n > self.max_batch:                     # bounded scratch and plan sizes
            return np.concatenate([self(u[i:i + self.max_batch]) for i in range(0, n, self.max_batch)])
        cap = max(self.min_bucket, 1 << (n - 1).bit_length())
        if cap not in self.buffers:
            self.buffers[cap] = (torch.empty((cap, 17), dtype=torch.float32, device=self.device),
                                 torch.empty(cap, dtype=torch.float64, device=self.device),
                                 np.zeros(cap, np.int32))
        tb, lb, sop = self.buffers[cap]
        th = self.theta(u)
        if n < cap:
            th = np.concatenate([th, np.repeat(th[:1], cap - n, axis=0)])
        t0 = time.perf_counter()
        tb.copy_(torch.from_numpy(th))
        binding.loglike_batch(tb, sop, [self.system], out=lb, ctx=self.ctx)
        out = lb[:n].cpu().numpy().copy()
        self.gpu_s += time.perf_counter() - t0
        self.n_calls += 1
        self.n_points += n
        return out


class SurrogateScreen(Screen):
    """The trained network as the sampler's screen.

    The margin at a threshold L_min is ``sigmas`` x the RMS residual (prediction
    minus exact log L) of the calibration pairs whose exact log L is nearest
    L_min: the network's held-out pairs plus this run's own exact evaluations.
    A draw predicted below L_min - margin is discarded. A slice proposal
    predicted above L_min + ``trust_sigmas`` x that RMS counts as inside without
    an exact render (the chain's final point is always rendered).

    With ``quantile`` q the margins come from the tails instead: the residuals
    are heavy-tailed and skewed (the network over-predicts more often than it
    under-predicts), so the discard margin is ``safety`` x the q-quantile of
    (exact - prediction) and the inside margin ``safety`` x the q-quantile of
    (prediction - exact), over the ``quantile_window`` held-out pairs centred
    on L_min in log L order. Only held-out pairs enter: the run's own exact evaluations exclude
    the draws the screen discarded and would understate the under-prediction
    tail.

    With ``pool`` (the (u, log L) pairs of an earlier run of the same problem)
    the network is refitted every ``refit_every`` iterations on the pairs of the
    current contour region: pool pairs and this run's recent exact evaluations
    with log L >= L_min - band, band = max(band_min, band_frac (L_best - L_min)).
    The refit re-standardises the inputs to those pairs' spread, so the network
    resolves the narrow posterior that a fit over the whole prior cannot.
    """

    def __init__(self, surrogate: Surrogate, sigmas: float = 3.0, window: int = 200, floor: float = 0.1,
                 max_skips: int = 2000, keep: int = 65536, pool=None, refit_every: int = 10,
                 band_min: float = 50.0, band_frac: float = 0.5, refit_max: int = 60000, refit_steps: int = 300,
                 seed: int = 0, trust_sigmas: Optional[float] = None, quantile: Optional[float] = None,
                 safety: float = 1.25, quantile_window: int = 1000, refit_batch: int = 1024):
        self.surrogate = surrogate
        self.sigmas = sigmas
        self.trust_sigmas = sigmas if trust_sigmas is None else trust_sigmas
        self.quantile, self.safety, self.quantile_window = quantile, safety, quantile_window
        self.window = window
        self.floor = floor
        self.max_skips = max_skips
        self.keep = keep
        self.pool = None if pool is None else (np.asarray(pool[0], np.float32), np.asarray(pool[1], np.float64))
        self.refit_every = refit_every
        self.band_min, self.band_frac = band_min, band_frac
        self.refit_max, self.refit_steps, self.refit_batch = refit_max, refit_steps, refit_batch
        self.rng = np.random.default_rng(seed)
        self.last_refit = None
        self.refits = []
        self._reset_calibration()
        self.run_u = np.zeros((0, 0), np.float32)
        self.run_ll = np.zeros(0)
        self.n_predicted = 0

    def _reset_calibration(self):
        self.held_l, self.held_r = (np.asarray(a, np.float64) for a in self.surrogate.margin_table)
        self.run_l = np.zeros(0)
        self.run_r = np.zeros(0)
        self._sorted = None

    def predict(self, u: np.ndarray) -> np.ndarray:
        self.n_predicted += len(u)
        return self.surrogate.predict(u)

    def observe(self, u: np.ndarray, exact: np.ndarray) -> None:
        """Add the residuals of exactly evaluated points to the calibration set
        (and the points to the refit data)."""
        ok = np.isfinite(exact)
        if not ok.any():
            return
        uu = np.asarray(u)[ok]
        pred = self.surrogate.predict(uu)
        ex = np.asarray(exact, np.float64)[ok]
        self.run_l = np.concatenate([self.run_l, ex])[-self.keep:]
        self.run_r = np.concatenate([self.run_r, pred - ex])[-self.keep:]
        if self.pool is not None:
            self.run_u = (uu.astype(np.float32) if self.run_u.size == 0
                          else np.concatenate([self.run_u, uu.astype(np.float32)])[-self.keep:])
            self.run_ll = np.concatenate([self.run_ll, ex])[-self.keep:]
        self._sorted = None

    def begin_iteration(self, lmin: float, it: int) -> None:
        if self.pool is None or (self.last_refit is not None and it - self.last_refit < self.refit_every):
            return
        pu, pl = self.pool
        best = max(float(pl.max()), float(self.run_ll.max()) if self.run_ll.size else -np.inf)
        band = max(self.band_min, self.band_frac * (best - lmin))
        sel_p = pl >= lmin - band
        u = pu[sel_p]
        ll = pl[sel_p]
        if self.run_ll.size:
            sel_r = self.run_ll >= lmin - band
            u = np.concatenate([u, self.run_u[sel_r]])
            ll = np.concatenate([ll, self.run_ll[sel_r]])
        if len(ll) < 2000:
            return
        if len(ll) > self.refit_max:
            pick = self.rng.choice(len(ll), self.refit_max, replace=False)
            u, ll = u[pick], ll[pick]
        info = self.surrogate.refit(u, ll, steps=self.refit_steps, batch=self.refit_batch, seed=it)
        info.update({"it": it, "lmin": lmin, "band": band})
        self.refits.append(info)
        self.last_refit = it
        self._reset_calibration()

    def get_state(self) -> dict:
        """Everything a resumed run needs: the (possibly refitted) network and the calibration."""
        sur = self.surrogate
        return {"params": sur.params.cpu().numpy(), "norm": sur.norm.cpu().numpy(), "l_ref": sur.l_ref,
                "mu": sur.mu, "P": sur.P,
                "table": sur.margin_table, "held": (self.held_l, self.held_r), "run": (self.run_l, self.run_r),
                "run_pairs": (self.run_u, self.run_ll), "last_refit": self.last_refit, "refits": self.refits,
                "rng": self.rng.bit_generator.state}

    def set_state(self, d: dict) -> None:
        sur = self.surrogate
        sur.params = torch.from_numpy(d["params"]).to(sur.device)
        sur.norm = torch.from_numpy(d["norm"]).to(sur.device)
        sur.l_ref, sur.margin_table = d["l_ref"], d["table"]
        sur.mu, sur.P = d["mu"], d["P"]
        self.held_l, self.held_r = d["held"]
        self.run_l, self.run_r = d["run"]
        self.run_u, self.run_ll = d["run_pairs"]
        self.last_refit, self.refits = d["last_refit"], d["refits"]
        self.rng.bit_generator.state = d["rng"]
        self._sorted = None

    def _rms(self, lmin: float) -> float:
        if self._sorted is None:
            ll = np.concatenate([self.held_l, self.run_l])
            order = np.argsort(ll)
            self._sorted = (ll[order], np.concatenate([self.held_r, self.run_r])[order])
        ll, res = self._sorted
        i = int(np.searchsorted(ll, lmin))
        lo, hi = max(0, i - self.window // 2), min(len(ll), i + self.window // 2)
        w = res[lo:hi] if hi > lo else res
        return float(np.sqrt(np.mean(w * w)))

    def _tail(self, lmin: float, sign: float) -> float:
        ll, res = self.held_l, self.held_r          # sorted by exact log L
        i = int(np.searchsorted(ll, lmin))
        h = self.quantile_window // 2
        lo, hi = max(0, i - h), min(len(ll), i + h)
        if hi - lo < self.quantile_window:           # near an end of the table: take the window whole
            lo, hi = max(0, hi - self.quantile_window), min(len(ll), lo + self.quantile_window)
        w = sign * res[lo:hi]
        return self.safety * float(np.quantile(w, self.quantile)) if len(w) else np.inf

    def margin(self, lmin: float) -> float:
        if self.quantile is not None:
            return max(self._tail(lmin, -1.0), self.floor)
        return max(self.sigmas * self._rms(lmin), self.floor)

    def margin_in(self, lmin: float) -> float:
        if self.quantile is not None:
            return max(self._tail(lmin, 1.0), self.floor)
        return max(self.trust_sigmas * self._rms(lmin), self.floor)


class _Observed:
    """The likelihood callable of a screened run: also feeds residuals back to the screen."""

    def __init__(self, loglike, screen: SurrogateScreen):
        self.loglike = loglike
        self.screen = screen

    def __call__(self, u):
        ll = self.loglike(u)
        self.screen.observe(u, ll)
        return ll


def _summary(res: NSResult, wall: float) -> dict:
    return {"logz": res.logz, "logz_err": res.logz_err, "n_exact": res.n_exact, "n_accepted": res.n_accepted,
            "n_iter": res.n_iter, "renders_per_accepted": res.renders_per_accepted,
            "n_screened_out": res.n_screened_out, "n_audit": res.n_audit, "n_false_reject": res.n_false_reject,
            "n_trusted": res.n_trusted, "n_false_accept": res.n_false_accept, "n_fallback": res.n_fallback,
            "converged": res.converged, "wall_s": wall}


class Suspended(Exception):
    """A run reached the deadline; its checkpoint is in the state directory."""


_ARRAYS = ("samples", "logl", "weights", "evaluated_u", "evaluated_logl")
_SCALARS = ("logz", "logz_err", "n_exact", "n_accepted", "n_iter", "n_screened_out", "n_audit", "n_false_reject",
            "n_trusted", "n_false_accept", "n_fallback", "converged")


def _save_result(path: str, res: NSResult, wall: float) -> None:
    arrays = {k: getattr(res, k) for k in _ARRAYS if getattr(res, k) is not None}
    arrays.update({k: np.asarray(getattr(res, k)) for k in _SCALARS})
    np.savez(path, wall=np.asarray(wall), **arrays)


def _load_result(path: str):
    with np.load(path) as z:
        kw = {k: z[k] for k in _ARRAYS if k in z.files}
        kw.update({k: z[k].item() for k in _SCALARS})
        return NSResult(**kw), float(z["wall"])


class ScreenExperiment:
    """Plain run A (records exact pairs), plain run B (another seed: the sampler's
    own spread), the surrogate trained on A's pairs, and the screened run C, each
    computed on first use and kept.

    With ``state_dir`` every finished run is saved there and reused by a later
    call, and a run still going at ``deadline`` (time.monotonic()) is
    checkpointed there and Suspended is raised; calling again resumes it."""

    def __init__(self, spec: SystemSpec, obs: Observation, device: torch.device, n_live: int = 400,
                 k_replace: int = 40, seeds=(5, 6, 7), dlogz: float = 0.5, max_iter: int = 5000,
                 train_epochs: int = 60, train_batch: int = 1024, sigmas: float = 3.0, log=print,
                 log_every: int = 100, record_per_iter: Optional[int] = 200, audit: float = 0.0,
                 state_dir: Optional[str] = None, deadline: Optional[float] = None, chunk: int = 25,
                 local: bool = True, refit_every: int = 5, refit_steps: int = 400, band_min: float = 25.0,
                 floor: float = 0.1, trust_sigmas: float = 3.0, quantile: Optional[float] = None,
                 safety: float = 1.25, refit_batch: int = 4096):
        self.spec, self.obs, self.device = spec, obs, device
        self.n_live, self.k_replace, self.seeds, self.dlogz, self.max_iter = n_live, k_replace, seeds, dlogz, max_iter
        self.train_epochs, self.train_batch = train_epochs, train_batch
        self.sigmas, self.trust_sigmas, self.floor = sigmas, trust_sigmas, floor
        self.quantile, self.safety, self.refit_batch = quantile, safety, refit_batch
        self.log, self.log_every, self.record_per_iter, self.audit = log, log_every, record_per_iter, audit
        self.state_dir, self.deadline, self.chunk = state_dir, deadline, chunk
        self.local, self.refit_every, self.refit_steps, self.band_min = local, refit_every, refit_steps, band_min
        self.ll = GpuLogLike(spec, obs, device)
        self.ndim = len(self.ll.free)
        self._runs: Dict[str, tuple] = {}
        self._sur = None
        self._screen = None

    def _path(self, name):
        import os
        return os.path.join(self.state_dir, name) if self.state_dir else None

    def _run(self, name, seed, screen=None, record=False, fn=None):
        import os
        sd, log = self.state_dir, self.log
        if sd and os.path.exists(self._path(name + ".npz")):
            log(f"{name}: loaded from {self._path(name + '.npz')}")
            return _load_result(self._path(name + ".npz"))
        s = NestedSampler(fn or self.ll, self.ndim, n_live=self.n_live, k_replace=self.k_replace, dlogz=self.dlogz,
                          seed=seed, max_iter=self.max_iter, record=record, record_per_iter=self.record_per_iter,
                          audit=self.audit if screen is not None else 0.0, audit_seed=seed, audit_loglike=self.ll)
        wall0 = 0.0
        if sd and os.path.exists(self._path(name + ".ckpt")):
            with open(self._path(name + ".ckpt"), "rb") as f:
                s.restore(f.read())
            wall0 = s.state.get("wall", 0.0)
            if isinstance(screen, SurrogateScreen) and "screen_run" in s.state:
                screen.set_state(s.state["screen_run"])
            log(f"{name}: resumed at iteration {s.state['it']}")
        t0 = time.perf_counter()
        while True:
            r = s.run(screen=screen, max_iter=self.chunk, log=log, log_every=self.log_every)
            if r.converged or r.n_iter >= self.max_iter:
                break
            if self.deadline is not None and time.monotonic() > self.deadline:
                if sd:
                    s.state["wall"] = wall0 + time.perf_counter() - t0
                    if isinstance(screen, SurrogateScreen):
                        s.state["screen_run"] = screen.get_state()
                    with open(self._path(name + ".ckpt"), "wb") as f:
                        f.write(s.checkpoint())
                raise Suspended(f"{name} suspended at iteration {r.n_iter}")
        wall = wall0 + time.perf_counter() - t0
        if sd:
            _save_result(self._path(name + ".npz"), r, wall)
        return r, wall

    def plain(self):
        """Run A, which records the exact pairs: (NSResult, wall seconds)."""
        if "a" not in self._runs:
            self.log(f"plain run A, seed {self.seeds[0]} (recording pairs)")
            ra, wa = self._runs["a"] = self._run("plain_a", self.seeds[0], record=True)
            self.log(f"  {ra.n_exact} exact evaluations, {ra.n_iter} iterations, log Z {ra.logz:.2f}, {wa:.1f} s")
        return self._runs["a"]

    def null(self):
        """Run B, another seed."""
        if "b" not in self._runs:
            self.log(f"plain run B, seed {self.seeds[1]}")
            rb, wb = self._runs["b"] = self._run("plain_b", self.seeds[1])
            self.log(f"  {rb.n_exact} exact evaluations, {rb.n_iter} iterations, log Z {rb.logz:.2f}, {wb:.1f} s")
        return self._runs["b"]

    def surrogate(self):
        """The network fitted on run A's pairs: (Surrogate, fit summary)."""
        import os
        if self._sur is None:
            ra, _ = self.plain()
            sur = Surrogate(self.device, seed=self.seeds[0], free=self.ll.free)
            if self.state_dir and os.path.exists(self._path("surrogate.npz")):
                fit = sur.load(self._path("surrogate.npz"))
                self.log("surrogate: loaded")
            else:
                t0 = time.perf_counter()
                fit = sur.fit(ra.evaluated_u, ra.evaluated_logl, epochs=self.train_epochs, batch=self.train_batch)
                torch.cuda.synchronize(self.device)
                fit["wall_s"] = time.perf_counter() - t0
                if self.state_dir:
                    sur.save(self._path("surrogate.npz"), fit)
            self.log(f"surrogate trained on {fit['n_train']} pairs in {fit['wall_s']:.1f} s, held-out rmse(y) "
                     f"{fit['rmse_y']:.4f}")
            self._sur = (sur, fit)
        return self._sur

    def _make_screen(self, sur, seed):
        ra, _ = self.plain()
        return SurrogateScreen(
            sur, sigmas=self.sigmas, pool=(ra.evaluated_u, ra.evaluated_logl) if self.local else None,
            seed=seed, refit_every=self.refit_every, refit_steps=self.refit_steps,
            band_min=self.band_min, floor=self.floor, trust_sigmas=self.trust_sigmas, quantile=self.quantile,
            safety=self.safety, refit_batch=self.refit_batch)

    def screened(self):
        """Run C, screened by the network (refitted locally when ``local``)."""
        if "c" not in self._runs:
            ra, _ = self.plain()
            sur, _ = self.surrogate()
            self._screen = self._make_screen(sur, self.seeds[2])
            self.log(f"screened run C, seed {self.seeds[2]}" +
                     (f" (network refitted locally every {self.refit_every} iterations)" if self.local else ""))
            rc, wc = self._runs["c"] = self._run("screened_c", self.seeds[2], screen=self._screen,
                                                 fn=_Observed(self.ll, self._screen))
            self.log(f"  {rc.n_exact} exact evaluations, {rc.n_screened_out} screened out, log Z {rc.logz:.2f}, "
                     f"{wc:.1f} s")
        return self._runs["c"]

    def summary(self, null: bool = True) -> dict:
        """Every stage (run on first use) and the comparison: renders per accepted
        point, evidences, posterior means and their shifts in plain-run sigmas."""
        ra, wa = self.plain()
        if null:
            rb, wb = self.null()
        _, fit = self.surrogate()
        rc, wc = self.screened()
        ll = self.ll
        to_theta = lambda u: ll.theta(u)[:, ll.free].astype(np.float64)
        ma, sa = ra.posterior_moments(to_theta)
        mc, sc = rc.posterior_moments(to_theta)
        out = {"system": self.spec.name, "n_live": self.n_live, "k_replace": self.k_replace, "ndim": self.ndim,
               "free": ll.free.tolist(), "audit_fraction": self.audit,
               "plain": _summary(ra, wa), "screened": _summary(rc, wc), "fit": fit,
               "renders_per_accepted_ratio": ra.renders_per_accepted / rc.renders_per_accepted,
               "posterior_mean_plain": ma.tolist(), "posterior_std_plain": sa.tolist(),
               "posterior_mean_screened": mc.tolist(), "posterior_std_screened": sc.tolist(),
               "shift_screened_sigma": (np.abs(mc - ma) / sa).tolist(),
               "settings": {"sigmas": self.sigmas, "trust_sigmas": self.trust_sigmas, "quantile": self.quantile,
                            "safety": self.safety, "floor": self.floor,
                            "refit_every": self.refit_every, "refit_steps": self.refit_steps,
                            "refit_batch": self.refit_batch,
                            "band_min": self.band_min, "local": self.local},
               "n_pairs_recorded": int(0 if ra.evaluated_u is None else len(ra.evaluated_u)),
               "refits": self._screen.refits if self._screen is not None else []}
        out["max_shift_screened_sigma"] = float(np.max(out["shift_screened_sigma"]))
        if null:
            mb, sb = rb.posterior_moments(to_theta)
            out.update({"plain_null": _summary(rb, wb), "posterior_mean_null": mb.tolist(),
                        "posterior_std_null": sb.tolist(), "shift_null_sigma": (np.abs(mb - ma) / sa).tolist()})
            out["max_shift_null_sigma"] = float(np.max(out["shift_null_sigma"]))
        return out


    def study(self, null_seeds, screened_seeds) -> dict:
        """The sampler's own spread and the screen's effect over several seeds.

        Plain runs with ``null_seeds`` give the null: how far a plain posterior
        mean lands from run A's by sampling noise alone. Screened runs with
        ``screened_seeds`` each start from the same network trained on run A's
        pairs (refits are undone between runs). Shifts are |mean - mean_A| in
        units of run A's posterior sigma, per parameter; each run is summarised
        by its largest shift. The render ratio of a screened run is the mean
        exact renders per accepted point of all plain runs (A and the nulls)
        over its own."""
        ra, wa = self.plain()
        sur, fit = self.surrogate()
        snap = sur.snapshot()
        ll = self.ll
        to_theta = lambda u: ll.theta(u)[:, ll.free].astype(np.float64)
        ma, sa = ra.posterior_moments(to_theta)

        def shifts(r):
            m, _ = r.posterior_moments(to_theta)
            return np.abs(m - ma) / sa

        nulls, screened = [], []
        for sd in null_seeds:
            self.log(f"plain run, seed {sd}")
            r, w = self._run(f"plain_s{sd}", sd)
            d = shifts(r)
            nulls.append(dict(_summary(r, w), seed=sd, shift_sigma=d.tolist(), max_shift_sigma=float(d.max())))
            self.log(f"  {r.n_exact} exact, log Z {r.logz:.2f}, largest shift {d.max():.3f} sigma, {w:.0f} s")
        plain_rpa = float(np.mean([ra.renders_per_accepted] + [n["renders_per_accepted"] for n in nulls]))
        for sd in screened_seeds:
            sur.restore(snap)
            screen = self._make_screen(sur, sd)
            self.log(f"screened run, seed {sd}")
            r, w = self._run(f"screened_s{sd}", sd, screen=screen, fn=_Observed(self.ll, screen))
            d = shifts(r)
            screened.append(dict(_summary(r, w), seed=sd, shift_sigma=d.tolist(), max_shift_sigma=float(d.max()),
                                 renders_per_accepted_ratio=plain_rpa / r.renders_per_accepted))
            self.log(f"  {r.n_exact} exact, ratio {plain_rpa / r.renders_per_accepted:.2f}, log Z {r.logz:.2f}, "
                     f"largest shift {d.max():.3f} sigma, {w:.0f} s")
        sur.restore(snap)
        null_max = [n["max_shift_sigma"] for n in nulls]
        scr_max = [c["max_shift_sigma"] for c in screened]
        ratios = [c["renders_per_accepted_ratio"] for c in screened]
        return {"system": self.spec.name, "n_live": self.n_live, "k_replace": self.k_replace, "ndim": self.ndim,
                "plain_a": dict(_summary(ra, wa), seed=self.seeds[0]), "fit": fit,
                "plain_renders_per_accepted_mean": plain_rpa, "null": nulls, "screened": screened,
                "null_max_shift_sigma": null_max, "screened_max_shift_sigma": scr_max,
                "renders_per_accepted_ratio": ratios, "ratio_mean": float(np.mean(ratios)) if ratios else None,
                "settings": {"sigmas": self.sigmas, "trust_sigmas": self.trust_sigmas, "quantile": self.quantile,
                             "safety": self.safety, "floor": self.floor, "refit_every": self.refit_every,
                             "refit_steps": self.refit_steps, "refit_batch": self.refit_batch,
                             "band_min": self.band_min, "local": self.local}}


def compare_runs(spec: SystemSpec, obs: Observation, device: torch.device, null: bool = True, **settings) -> dict:
    """The whole experiment in one call (ScreenExperiment's settings as keywords)."""
    return ScreenExperiment(spec, obs, device, **settings).summary(null=null)


def library_mock(spec: SystemSpec, device: torch.device) -> Observation:
    """A mock observation of spec whose noiseless image the library itself renders."""
    from .mocks import make_observation
    psf = torch.from_numpy(spec.psf).to(device)
    rsys = binding.System(psf, pixscale=spec.pixscale, nsub=spec.nsub, height=spec.height, width=spec.width,
                          center=(spec.center_x, spec.center_y))
    return make_observation(
        spec, lambda t: binding.render(torch.from_numpy(np.asarray(t, np.float32)).to(device), rsys).cpu().numpy())


def main(argv=None) -> int:
    import argparse
    import json
    import os
    import sys

    from . import mocks
    ap = argparse.ArgumentParser(description="nested sampling with and without the learned screen")
    ap.add_argument("--system", choices=["64x64", "200x200"], default="200x200")
    ap.add_argument("--n-live", type=int, default=400)
    ap.add_argument("--k-replace", type=int, default=40)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--sigmas", type=float, default=3.0)
    ap.add_argument("--quantile", type=float, default=None,
                    help="margins from this quantile of the held-out residual tails (else sigmas x RMS)")
    ap.add_argument("--safety", type=float, default=1.25, help="factor on the quantile margins")
    ap.add_argument("--trust-sigmas", type=float, default=3.0,
                    help="slice proposals predicted this many residual RMS above the threshold skip the render")
    ap.add_argument("--refit-every", type=int, default=5)
    ap.add_argument("--refit-steps", type=int, default=400)
    ap.add_argument("--refit-batch", type=int, default=4096)
    ap.add_argument("--max-iter", type=int, default=5000)
    ap.add_argument("--audit", type=float, default=0.0, help="fraction of screened-out draws also evaluated exactly")
    ap.add_argument("--state-dir", default=None, help="save finished runs and checkpoints here; resume from it")
    ap.add_argument("--time-limit", type=float, default=None, help="seconds before the running stage is suspended")
    ap.add_argument("--out", default=None)
    ap.add_argument("--null-seeds", type=int, nargs="*", default=None,
                    help="seed study: plain runs with these seeds (the null spread about run A)")
    ap.add_argument("--screened-seeds", type=int, nargs="*", default=None,
                    help="seed study: screened runs with these seeds, each from the network trained on run A")
    a = ap.parse_args(argv)
    if not torch.cuda.is_available():
        print("a GPU is required", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    spec = mocks.c0_spec() if a.system == "64x64" else mocks.c1_spec()
    obs = library_mock(spec, dev)
    log = lambda m: print(m, flush=True)
    if a.state_dir:
        os.makedirs(a.state_dir, exist_ok=True)
    deadline = time.monotonic() + a.time_limit if a.time_limit else None
    settings = dict(n_live=a.n_live, k_replace=a.k_replace, train_epochs=a.epochs, sigmas=a.sigmas,
                    max_iter=a.max_iter, seeds=(mocks.C4_SEED, mocks.C4_SEED + 1, mocks.C4_SEED + 2), log=log,
                    audit=a.audit, state_dir=a.state_dir, deadline=deadline, trust_sigmas=a.trust_sigmas,
                    refit_every=a.refit_every, refit_steps=a.refit_steps, quantile=a.quantile, safety=a.safety,
                    refit_batch=a.refit_batch)
    try:
        if a.null_seeds is not None or a.screened_seeds is not None:
            res = ScreenExperiment(spec, obs, dev, **settings).study(a.null_seeds or [], a.screened_seeds or [])
        else:
            res = compare_runs(spec, obs, dev, **settings)
    except Suspended as e:
        print(f"suspended: {e}", flush=True)
        return 3
    text = json.dumps(res)
    print(text, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text + "\n")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
