"""lensed_loglike_noalloc (the allocation-free plain log L) against
lensed_loglike, through the C ABI: two calls in a row on the same device, the
second with a smaller image, each equal to the context path bit for bit; sizes
beyond the static workspace are refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1505_07674_amd as lensed
from paper_1505_07674_amd import mocks
from paper_1505_07674_amd.binding import LensedSystemC, lib

from helpers import observation
from test_gpu_parity import _custom_spec, gpu_system

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
LENSED_TOO_LARGE = 5


def noalloc(theta, system):
    f = lib().lensed_loglike_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(LensedSystemC), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    out = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    t = theta.contiguous()
    rc = f(ctypes.byref(system.c_struct), ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(out.data_ptr()),
           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, out


def test_noalloc_matches_the_context_path_twice_then_smaller():
    big_spec, big_obs = observation("c1")
    small = _custom_spec(37, 53, 3, mocks.moffat_psf(7, 0.1, 3.0))
    rng = np.random.default_rng(2)
    small_obs = mocks.Observation(small, rng.standard_normal((37, 53)).astype(np.float32),
                                  (rng.random((37, 53)) < 0.7).astype(np.float32) * 10.0, 0.3)
    cases = [(big_spec, big_obs, mocks.points(big_spec, 2, seed=91)),
             (small, small_obs, mocks.points(small, 2, seed=92))]
    for spec, obs, pts in cases:
        gs = gpu_system(spec, obs)
        for t in pts:
            tt = torch.from_numpy(t).to(DEV)
            ref = lensed.loglike(tt, gs).cpu().numpy()[0]
            rc, out = noalloc(tt, gs)
            assert rc == 0, lib().lensed_status_string(rc)
            got = out.cpu().numpy()[0]
            print(f"{spec.name}: noalloc {got!r} context {ref!r}", flush=True)
            assert np.isfinite(ref) and got == ref


def test_noalloc_refuses_images_beyond_the_workspace():
    big = lensed.System(torch.ones((3, 3), device=DEV), torch.zeros((2048, 2048), device=DEV),
                        torch.ones((2048, 2048), device=DEV), pixscale=0.05, nsub=1)
    rc, out = noalloc(torch.from_numpy(mocks.c1_spec().truth).to(DEV), big)
    assert rc == LENSED_TOO_LARGE
    assert torch.isnan(out).all()
