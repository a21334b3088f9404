"""Masked batches (lensed_loglike_batch_masked): only the pixels Eq. 17 can see
are rendered (the w > 0 support dilated by the PSF box of Eq. 15, clamped at
the borders) and only PSF tiles holding a pixel with w > 0 are convolved. Masking
is w = 0 (Sec. 3.2), so the result must equal the all-pixel batch bit for bit,
and the FP64 oracle to the usual bar."""
import numpy as np
import pytest
import torch

import oracle
import paper_1505_07674_amd as lensed
from paper_1505_07674_amd import mocks
from paper_1505_07674_amd.binding import Context

from helpers import golden, golden_file, loglike_tolerance, observation, oracle_loglikes, oracle_system
from test_gpu_parity import _custom_spec, gpu_system

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def test_c1_masked_equals_all_pixels_and_the_oracle():
    spec, obs = observation("c1")
    pts = golden.c1_points(spec)[:512]
    gold = golden_file(golden.C1_FILE)["loglike"][:512]
    gs = gpu_system(spec, obs)
    tp = torch.from_numpy(pts).to(DEV)
    sop = np.zeros(len(pts), np.int32)
    ctx = Context(0)
    full = lensed.loglike_batch(tp, sop, [gs], ctx=ctx).cpu().numpy()
    all_px = ctx.batch_rendered()
    masked = lensed.loglike_batch(tp, sop, [gs], ctx=ctx, masked=True).cpu().numpy()
    vis = ctx.batch_rendered()
    ctx.close()
    say(f"rendered pixels per launch: all {all_px['pixels']}, masked {vis['pixels']} "
        f"({vis['pixels'] / all_px['pixels']:.3f})")
    assert all_px["pixels"] == 512 * 200 * 200
    assert vis["pixels"] < 0.6 * all_px["pixels"]
    assert np.array_equal(masked, full)
    assert np.all(np.abs(masked - gold) <= loglike_tolerance(gold, obs.weight))


@pytest.mark.parametrize("ppt", [1, 2])
def test_masked_mixed_shapes_equal_all_pixels(ppt, monkeypatch):
    """Random masks on mixed shapes: odd widths, masks touching the borders, a
    system with no weighted pixel, several N and a Gauss-Kronrod rule."""
    monkeypatch.setenv("LENSED_RENDER_PPT", str(ppt))
    rng = np.random.default_rng(5 + ppt)
    shapes = [(50, 64, 4, 21, "sub"), (37, 53, 3, 7, "sub"), (64, 64, 2, 7, "sub"), (20, 31, 7, 5, "g3k7"),
              (40, 40, 2, 9, "sub")]
    systems, pts_all, sop = [], [], []
    for s, (H, W, N, P, rule) in enumerate(shapes):
        spec = _custom_spec(H, W, N, mocks.moffat_psf(P, 0.1, 3.0))
        model = oracle.render(oracle_system(spec), spec.truth.astype(np.float64))
        data = (model + 0.01 * rng.standard_normal(model.shape)).astype(np.float32)
        w = np.zeros((H, W), np.float32)
        if s == 0:
            w[5:12, 40:64] = 1e4                      # touches the right border
        elif s == 1:
            w[rng.random((H, W)) < 0.02] = 1e4        # scattered pixels
        elif s == 2:
            w[20:44, 20:44] = 1e4                     # a block in the middle
        elif s == 3:
            w[0, 0] = 1e4                             # one corner pixel
        # s == 4: nothing weighted
        g = gpu_system(spec, mocks.Observation(spec, data, w, 0.01))
        if rule != "sub":
            g = lensed.System(g.psf, g.data, g.weight, pixscale=spec.pixscale, nsub=N, height=H, width=W,
                              center=(spec.center_x, spec.center_y), rule=rule)
        systems.append(g)
        pts_all.append(mocks.points(spec, 16, seed=40 + s))
        sop.append(np.full(16, s, np.int32))
    tp = torch.from_numpy(np.concatenate(pts_all)).to(DEV)
    sop = np.concatenate(sop)
    ctx = Context(0)
    full = lensed.loglike_batch(tp, sop, systems, ctx=ctx).cpu().numpy()
    masked = lensed.loglike_batch(tp, sop, systems, ctx=ctx, masked=True).cpu().numpy()
    # a second call replays the cached masked plan: same values
    again = lensed.loglike_batch(tp, sop, systems, ctx=ctx, masked=True).cpu().numpy()
    ctx.close()
    assert np.all(np.isfinite(full))
    assert np.array_equal(masked, full), np.max(np.abs(masked - full))
    assert np.array_equal(again, masked)
    assert np.all(full[sop == 4] == 0.0)
