"""Render schedules of the batch engine (the batching of Eq. 17 over points and
systems): one pixel per thread, or two horizontally adjacent pixels per thread
sharing the row terms of the subsample grid, in blocks of 128, 256 or 512
threads. Each pixel is computed by the same
operations on the same constants either way, so the batched log L must agree
bit for bit between the schedules, and with the FP64 oracle to the usual bar.
Systems of odd width, and the Gauss-Kronrod classes, keep one pixel per thread
inside the same launch."""
import os

import numpy as np
import pytest
import torch

import paper_1505_07674_amd as lensed
from paper_1505_07674_amd import mocks
from paper_1505_07674_amd.binding import Context

from helpers import loglike_tolerance, oracle_loglikes, oracle_system
from test_gpu_parity import _custom_spec, gpu_system

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def context_with(ppt, block=256):
    """A context with the render schedule fixed and the PSF tile left to the
    cost model: two contexts autotuning by timing could pick different PSF
    tiles, whose chi^2 partial sums group the pixels differently."""
    env = {"LENSED_RENDER_PPT": str(ppt), "LENSED_RENDER_BLOCK": str(block), "LENSED_NO_AUTOTUNE": "1"}
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


def mixed_systems():
    """Even and odd widths, several N, the point rule and a Gauss-Kronrod system."""
    rng = np.random.default_rng(11)
    shapes = [(60, 80, 4, "sub"), (37, 53, 3, "sub"), (41, 64, 2, "sub"), (30, 30, 1, "sub"), (24, 26, 7, "g3k7"),
              (33, 48, 8, "sub")]
    out = []
    for H, W, N, rule in shapes:
        psf = mocks.moffat_psf(7, 0.1, 3.0)
        spec = _custom_spec(H, W, N, psf)
        osys = oracle_system(spec)
        model = __import__("oracle").render(osys, spec.truth.astype(np.float64))
        obs = mocks.Observation(spec, (model + 0.01 * rng.standard_normal(model.shape)).astype(np.float32),
                                (rng.random(model.shape) < 0.9).astype(np.float32) * 1e4, 0.01)
        gs = gpu_system(spec, obs)
        if rule != "sub":
            gs = lensed.System(gs.psf, gs.data, gs.weight, pixscale=spec.pixscale, nsub=N, height=H, width=W,
                               center=(spec.center_x, spec.center_y), rule=rule)
        out.append((spec, obs, gs, rule))
    return out


def test_pair_schedule_is_bitwise_identical_and_matches_the_oracle():
    systems = mixed_systems()
    per = 24
    pts = np.concatenate([mocks.points(spec, per, seed=50 + i) for i, (spec, _, _, _) in enumerate(systems)])
    sop = np.repeat(np.arange(len(systems), dtype=np.int32), per)
    tp = torch.from_numpy(pts).to(DEV)
    gsys = [g for _, _, g, _ in systems]
    results = {}
    for ppt in (1, 2):
        ctx = context_with(ppt)
        results[ppt] = lensed.loglike_batch(tp, sop, gsys, ctx=ctx).cpu().numpy()
        sched = ctx.batch_schedule()
        say(f"render pixels per thread {ppt}: schedule {sched}")
        assert sched["render_pixels_per_thread"] == ppt
        ctx.close()
    assert np.all(np.isfinite(results[1]))
    assert np.array_equal(results[1], results[2]), np.max(np.abs(results[1] - results[2]))
    for i, (spec, obs, _, rule) in enumerate(systems):
        if rule != "sub":
            continue   # the Gauss-Kronrod oracle is checked in the rule tests
        sl = slice(i * per, (i + 1) * per)
        ref = oracle_loglikes(oracle_system(spec, obs), pts[sl])
        assert np.all(np.abs(results[1][sl] - ref) <= loglike_tolerance(ref, obs.weight)), spec.name


def test_c1_pair_schedule_matches_single_pixel_schedule():
    from helpers import observation
    spec, obs = observation("c1")
    pts = mocks.points(spec, 256, seed=21)
    tp = torch.from_numpy(pts).to(DEV)
    gs = gpu_system(spec, obs)
    out = {}
    for ppt in (1, 2):
        ctx = context_with(ppt)
        out[ppt] = lensed.loglike_batch(tp, np.zeros(len(pts), np.int32), [gs], ctx=ctx).cpu().numpy()
        ctx.close()
    assert np.array_equal(out[1], out[2])


@pytest.mark.parametrize("ppt", [1, 2])
def test_render_block_sizes_are_bitwise_identical(ppt):
    """Blocks of 128, 256 and 512 render threads cover the same units with the
    same arithmetic, so log L agrees bit for bit; the cusp list holds one entry
    per wave whatever the block, so the cusp-heavy mixed systems check it too."""
    systems = mixed_systems()
    per = 20
    pts = np.concatenate([mocks.points(spec, per, seed=80 + i) for i, (spec, _, _, _) in enumerate(systems)])
    sop = np.repeat(np.arange(len(systems), dtype=np.int32), per)
    tp = torch.from_numpy(pts).to(DEV)
    gsys = [g for _, _, g, _ in systems]
    out = {}
    for block in (128, 256, 512):
        ctx = context_with(ppt, block)
        out[block] = lensed.loglike_batch(tp, sop, gsys, ctx=ctx).cpu().numpy()
        sched = ctx.batch_schedule()
        say(f"ppt {ppt} block {block}: schedule {sched}")
        assert sched["render_block"] == block and sched["render_pixels_per_thread"] == ppt
        masked = lensed.loglike_batch(tp, sop, gsys, ctx=ctx, masked=True).cpu().numpy()
        assert np.array_equal(masked, out[block]), block
        ctx.close()
    assert np.all(np.isfinite(out[256]))
    assert np.array_equal(out[128], out[256]) and np.array_equal(out[512], out[256])


def test_autotuner_records_a_render_schedule():
    from helpers import observation
    spec, obs = observation("c0")
    pts = mocks.points(spec, 64, seed=3)
    ctx = Context(0)
    ll = lensed.loglike_batch(torch.from_numpy(pts).to(DEV), np.zeros(len(pts), np.int32), [gpu_system(spec, obs)],
                              ctx=ctx)
    torch.cuda.synchronize()
    sched = ctx.batch_schedule()
    say(f"autotuned schedule for 64x64 N=2: {sched}")
    assert sched["render_pixels_per_thread"] in (1, 2)
    assert sched["render_block"] in (128, 256, 512)
    assert sched["psf_tile"][0] > 0 and sched["psf_tile"][1] > 0
    assert torch.all(torch.isfinite(ll))
    ctx.close()


def test_gradient_plans_take_the_render_schedule():
    """A gradient plan renders with the schedule's pixels per thread while its
    gradient kernels keep their own one-pixel items: log L and gradient agree
    bit for bit between the schedules."""
    from test_gpu_grad import gpu_system as grad_system, small_obs, small_spec
    spec = small_spec(H=40, W=36, N=4)
    obs = small_obs(spec)
    gs = grad_system(spec, obs)
    pts = torch.from_numpy(mocks.points(spec, 12, seed=61)).to(DEV)
    out = {}
    for ppt, block in ((1, 256), (2, 256), (2, 512), (1, 128)):
        ctx = context_with(ppt, block)
        ll, g = lensed.loglike_grad(pts, gs, ctx=ctx)
        out[ppt, block] = (ll.cpu().numpy(), g.cpu().numpy())
        ctx.close()
    assert np.all(np.isfinite(out[1, 256][1]))
    for key in out:
        assert np.array_equal(out[1, 256][0], out[key][0]), key
        assert np.array_equal(out[1, 256][1], out[key][1]), key
