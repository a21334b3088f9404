"""Shared helpers for the parity tests: build the same seeded observation for the
oracle (float64 copies of float32 arrays) and for the GPU library."""
import functools
import importlib.util
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle
from paper_1505_07674_amd import mocks


def f32(x):
    return float(np.float32(x))


def oracle_system(spec, obs=None):
    data = None if obs is None else obs.data.astype(np.float64)
    weight = None if obs is None else obs.weight.astype(np.float64)
    return oracle.System(spec.height, spec.width, f32(spec.pixscale), spec.nsub, spec.psf.astype(np.float64),
                         data, weight, center_x=f32(spec.center_x), center_y=f32(spec.center_y))


@functools.lru_cache(maxsize=None)
def _observation(key):
    kind, idx = key
    spec = {"c0": mocks.c0_spec, "c1": mocks.c1_spec}[kind]() if kind != "c2" else mocks.c2_specs()[idx]
    osys = oracle_system(spec)
    obs = mocks.make_observation(spec, lambda t: oracle.render(osys, np.asarray(t, np.float64)))
    return spec, obs


def observation(kind, idx=0):
    """(spec, obs) of a standard workload, mock rendered by the oracle."""
    return _observation((kind, idx))


def oracle_loglikes(osys, thetas, threads=8):
    th = [np.asarray(t, np.float64) for t in thetas]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return np.array(list(ex.map(lambda t: oracle.loglike(osys, t), th)))


def loglike_tolerance(ll_ref, weight):
    """|delta log L| bound: 1e-6 relative, floored at the expected |log L| at the truth (N_w / 2)."""
    nw = int(np.count_nonzero(weight))
    return 1e-6 * np.maximum(np.abs(ll_ref), nw / 2.0)


def _load_golden_module():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "make_golden.py")
    spec = importlib.util.spec_from_file_location("make_golden", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


# the script that wrote the stored oracle values: its point generators and digests
golden = _load_golden_module()


def golden_file(path):
    """Arrays of a stored-values file (no pickles)."""
    with np.load(path, allow_pickle=False) as f:
        return {k: f[k] for k in f.files}
