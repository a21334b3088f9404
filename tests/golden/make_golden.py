"""Writes the oracle's expected values for the full-size parity tests.

Calls only the FP64 oracle (oracle/) and the seeded input generators
(paper_1505_07674_amd/mocks.py, which hold none of the method's arithmetic).
Nothing here touches the GPU library. Run on the CPU:

    python tests/golden/make_golden.py            # all three files
    python tests/golden/make_golden.py c1 c3      # a subset

Files (numpy .npz, no pickles; every file records sha256 digests of the inputs
it was computed from, so a test that rebuilds the inputs can prove they match):

  oracle_c1_loglike.npz  log L (Sec. 3.2 Eq. 17) of all 4096 points of the
                         200x200, 4x4-subsampled, 21x21-Moffat batch (point 0 is
                         the mock's truth), mock rendered by the oracle.
  oracle_c2_loglike.npz  log L of every point of the 16-system mixed batch
                         (16 x 512 = 8192 points; sides 64..300, N = 2..8).
  oracle_c3_grad.npz     log L and the exact 17-gradient (forward-mode dual
                         numbers through Eqs. 17, 15, 14, 2, 1) of every 8th
                         point of the 1024-point gradient batch (128 points,
                         point 0 is the truth).
"""
import hashlib
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1505_07674_amd import mocks  # noqa: E402

C1_FILE = os.path.join(HERE, "oracle_c1_loglike.npz")
C2_FILE = os.path.join(HERE, "oracle_c2_loglike.npz")
C3_FILE = os.path.join(HERE, "oracle_c3_grad.npz")
C1_POINTS = 4096
C2_POINTS_PER_SYSTEM = 512
C3_POINTS, C3_STRIDE = 1024, 8


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def f32(x):
    return float(np.float32(x))


def oracle_system(spec, obs=None):
    data = None if obs is None else obs.data.astype(np.float64)
    weight = None if obs is None else obs.weight.astype(np.float64)
    return oracle.System(spec.height, spec.width, f32(spec.pixscale), spec.nsub, spec.psf.astype(np.float64),
                         data, weight, center_x=f32(spec.center_x), center_y=f32(spec.center_y))


def oracle_observation(spec):
    osys = oracle_system(spec)
    return mocks.make_observation(spec, lambda t: oracle.render(osys, np.asarray(t, np.float64)))


def c1_points(spec):
    pts = mocks.points(spec, C1_POINTS, seed=mocks.C1_POINT_SEED)
    pts[0] = spec.truth
    return pts


def c2_points(spec, s):
    return mocks.points(spec, C2_POINTS_PER_SYSTEM, seed=mocks.C2_BASE_SEED * 100 + s)


def c3_points(spec):
    pts = mocks.points(spec, C3_POINTS, seed=mocks.C3_SEED)
    pts[0] = spec.truth
    return pts


def c3_index():
    return np.arange(0, C3_POINTS, C3_STRIDE)


def _map(fn, items, threads):
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))


def make_c1(threads):
    spec = mocks.c1_spec()
    obs = oracle_observation(spec)
    osys = oracle_system(spec, obs)
    pts = c1_points(spec)
    t0 = time.time()
    ll = np.array(_map(lambda t: oracle.loglike(osys, np.asarray(t, np.float64)), pts, threads))
    print(f"c1: {len(pts)} points in {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(C1_FILE, loglike=ll, theta_sha256=digest(pts), data_sha256=digest(obs.data),
                        weight_sha256=digest(obs.weight))


def make_c2(threads):
    specs = mocks.c2_specs()
    lls, tdig, ddig, wdig = [], [], [], []
    t0 = time.time()
    for s, spec in enumerate(specs):
        obs = oracle_observation(spec)
        osys = oracle_system(spec, obs)
        pts = c2_points(spec, s)
        lls.append(_map(lambda t: oracle.loglike(osys, np.asarray(t, np.float64)), pts, threads))
        tdig.append(digest(pts))
        ddig.append(digest(obs.data))
        wdig.append(digest(obs.weight))
        print(f"c2: system {s} ({spec.name}) done at {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(C2_FILE, loglike=np.array(lls), theta_sha256=np.array(tdig), data_sha256=np.array(ddig),
                        weight_sha256=np.array(wdig))


def make_c3(threads):
    spec = mocks.c1_spec()
    obs = oracle_observation(spec)
    osys = oracle_system(spec, obs)
    pts = c3_points(spec)
    idx = c3_index()
    t0 = time.time()
    res = _map(lambda t: oracle.loglike_grad(osys, np.asarray(t, np.float64)), pts[idx], threads)
    print(f"c3: {len(idx)} gradients in {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(C3_FILE, index=idx, loglike=np.array([r[0] for r in res]),
                        grad=np.array([r[1] for r in res]), theta_sha256=digest(pts),
                        data_sha256=digest(obs.data), weight_sha256=digest(obs.weight))


def main(argv):
    threads = min(len(os.sched_getaffinity(0)), 16)
    which = argv or ["c1", "c2", "c3"]
    for w in which:
        {"c1": make_c1, "c2": make_c2, "c3": make_c3}[w](threads)


if __name__ == "__main__":
    main(sys.argv[1:])
