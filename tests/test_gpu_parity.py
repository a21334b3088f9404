"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars (per point): on the model image L* (after the PSF) max |delta| <= 1e-5 x
peak |oracle pixel|, and |delta log L| <= 1e-6 x max(|log L_oracle|, N_w/2)
where N_w counts weighted pixels (the expected |log L| at the truth; avoids 0/0
for noiseless data). The unconvolved image L (render with apply_psf = 0) is
held to the same 1e-5 x peak bar as L*.

The full-size batches (all 4096 points of the 200x200 batch, all 8192 points of
the 16-system mixed batch) are compared point by point with oracle values
stored under tests/golden/ by tests/golden/make_golden.py, which calls only the
oracle; the stored input digests prove that the test rebuilt the same inputs.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_1505_07674_amd as lensed
from paper_1505_07674_amd import mocks

from helpers import f32, golden, golden_file, loglike_tolerance, observation, oracle_loglikes, oracle_system

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)


def gpu_system(spec, obs=None):
    data = None if obs is None else torch.from_numpy(obs.data).to(DEV)
    weight = None if obs is None else torch.from_numpy(obs.weight).to(DEV)
    return lensed.System(torch.from_numpy(spec.psf).to(DEV), data, weight, pixscale=spec.pixscale,
                         nsub=spec.nsub, height=spec.height, width=spec.width,
                         center=(spec.center_x, spec.center_y))


def check_images(spec, thetas, apply_psf, tol=1e-5):
    gsys = gpu_system(spec)
    osys = oracle_system(spec)
    errs = []
    for t in thetas:
        img = lensed.render(torch.from_numpy(t).to(DEV), gsys, apply_psf=apply_psf).cpu().numpy().astype(np.float64)
        ref = oracle.render(osys, t.astype(np.float64), apply_psf=apply_psf)
        errs.append(np.max(np.abs(img - ref)) / np.max(np.abs(ref)))
    errs = np.array(errs)
    say(f"  {spec.name} apply_psf={apply_psf}: worst pixel error {errs.max():.3e} x peak")
    worst = int(np.argmax(errs))
    assert errs.max() <= tol, f"pixel error {errs.max():.3e} x peak at theta={thetas[worst].tolist()}"
    return errs.max()


def test_c0_render_parity():
    spec, _ = observation("c0")
    say("c0 render parity")
    pts = mocks.points(spec, 24, seed=mocks.C0_POINT_SEED)
    check_images(spec, pts, True)
    check_images(spec, pts[:8], False)


def test_c0_loglike_batch_parity_all_points():
    spec, obs = observation("c0")
    say("c0 loglike batch, 1000 points")
    pts = mocks.points(spec, 1000, seed=mocks.C0_POINT_SEED)
    gsys = gpu_system(spec, obs)
    ll = lensed.loglike_batch(torch.from_numpy(pts).to(DEV), np.zeros(1000, np.int32), [gsys]).cpu().numpy()
    ref = oracle_loglikes(oracle_system(spec, obs), pts)
    tol = loglike_tolerance(ref, obs.weight)
    bad = np.nonzero(np.abs(ll - ref) > tol)[0]
    assert bad.size == 0, f"{bad.size} points off, e.g. {ll[bad[:3]]} vs {ref[bad[:3]]}"


def test_c0_plain_matches_batch_and_oracle():
    spec, obs = observation("c0")
    say("c0 plain loglike")
    pts = mocks.points(spec, 48, seed=11)
    gsys = gpu_system(spec, obs)
    tp = torch.from_numpy(pts).to(DEV)
    plain = torch.cat([lensed.loglike(tp[i], gsys) for i in range(len(pts))]).cpu().numpy()
    batch = lensed.loglike_batch(tp, np.zeros(len(pts), np.int32), [gsys]).cpu().numpy()
    ref = oracle_loglikes(oracle_system(spec, obs), pts)
    tol = loglike_tolerance(ref, obs.weight)
    assert np.all(np.abs(plain - ref) <= tol)
    assert np.all(np.abs(batch - ref) <= tol)
    assert np.all(np.abs(plain - batch) <= tol)


def test_c1_render_parity():
    spec, _ = observation("c1")
    say("c1 render parity")
    pts = np.concatenate([spec.truth[None, :], mocks.points(spec, 11, seed=mocks.C1_POINT_SEED)])
    check_images(spec, pts, True)
    check_images(spec, pts, False)


def test_c1_loglike_batch_parity_every_point():
    """The 4096-point batch the benchmark times, every point against the oracle."""
    spec, obs = observation("c1")
    say("c1 loglike batch, 4096 points, all compared")
    pts = golden.c1_points(spec)
    gold = golden_file(golden.C1_FILE)
    assert str(gold["theta_sha256"]) == golden.digest(pts), "C1 points differ from those of the stored values"
    assert str(gold["data_sha256"]) == golden.digest(obs.data), "C1 mock differs from the stored one"
    assert str(gold["weight_sha256"]) == golden.digest(obs.weight)
    ref = gold["loglike"]
    gsys = gpu_system(spec, obs)
    ll = lensed.loglike_batch(torch.from_numpy(pts).to(DEV), np.zeros(len(pts), np.int32), [gsys]).cpu().numpy()
    tol = loglike_tolerance(ref, obs.weight)
    ratio = np.abs(ll - ref) / tol
    say(f"  worst |delta log L| / bar = {ratio.max():.3f} at point {int(np.argmax(ratio))}")
    bad = np.nonzero(~(ratio <= 1.0))[0]
    assert bad.size == 0, f"{bad.size} of {len(pts)} points off, e.g. {bad[:5].tolist()}"


def test_profiled_stages_give_the_graph_result():
    """With profiling on, the batch runs stage by stage between hipEvents instead
    of as the captured graph: the same kernels, so the same log L bit for bit,
    and five stage times per call."""
    spec, obs = observation("c1")
    say("c1 loglike batch, 512 points, graph vs profiled stages")
    pts = torch.from_numpy(mocks.points(spec, 512, seed=mocks.C1_POINT_SEED + 5)).to(DEV)
    gsys = gpu_system(spec, obs)
    sop = np.zeros(512, np.int32)
    ctx = lensed.Context(0)
    a = lensed.loglike_batch(pts, sop, [gsys], ctx=ctx).cpu().numpy()
    ctx.set_profiling(True)
    ctx.stage_times()
    b = lensed.loglike_batch(pts, sop, [gsys], ctx=ctx).cpu().numpy()
    b2 = lensed.loglike_batch(pts, sop, [gsys], ctx=ctx).cpu().numpy()
    stages, calls = ctx.stage_times()
    ctx.set_profiling(False)
    assert np.array_equal(a, b) and np.array_equal(a, b2)
    assert calls == 2 and tuple(stages) == lensed.Context.STAGES
    assert all(v >= 0.0 for v in stages.values()) and stages["render"] > 0.0 and stages["psf_chi2"] > 0.0
    c = lensed.loglike_batch(pts, sop, [gsys], ctx=ctx).cpu().numpy()
    assert np.array_equal(a, c)


def test_c1_plain_matches_oracle():
    spec, obs = observation("c1")
    say("c1 plain loglike")
    pts = mocks.points(spec, 6, seed=21)
    gsys = gpu_system(spec, obs)
    tp = torch.from_numpy(pts).to(DEV)
    plain = torch.cat([lensed.loglike(tp[i], gsys) for i in range(len(pts))]).cpu().numpy()
    ref = oracle_loglikes(oracle_system(spec, obs), pts)
    assert np.all(np.abs(plain - ref) <= loglike_tolerance(ref, obs.weight))


def _custom_spec(H, W, N, psf, pixscale=0.07, center=(0.1, -0.05)):
    base = mocks.c1_spec()
    return mocks.SystemSpec(f"custom_{H}x{W}_sub{N}", H, W, N, psf.astype(np.float32), base.truth, base.prior,
                            np.ones((H, W), bool), 77, False, pixscale=pixscale, center_x=center[0],
                            center_y=center[1])


@pytest.mark.parametrize("H,W,N,ph,pw", [
    (37, 53, 3, 5, 9),       # ragged tiles, generic stencil, odd N
    (64, 64, 1, 1, 1),       # point rule, no blurring
    (1, 1, 2, 3, 3),         # single pixel
    (5, 129, 5, 7, 7),       # thin strip, specialised 7x7 stencil
    (90, 33, 16, 21, 21),    # largest N, specialised 21x21 stencil, ragged
    (20, 20, 9, 3, 5),       # N outside the specialised set
    (77, 170, 2, 21, 21),    # wide 21x21 tiles, ragged rows
    (45, 236, 2, 21, 21),    # the widest single wide tile
    (50, 237, 2, 21, 21),    # wide tiles, two or three per row
])
def test_ragged_and_generic_shapes(H, W, N, ph, pw):
    say(f"shape {H}x{W} N={N} psf {ph}x{pw}")
    rng = np.random.default_rng(H * 1000 + W)
    psf = rng.random((ph, pw)) + 0.1
    spec = _custom_spec(H, W, N, psf)
    pts = mocks.points(spec, 3, seed=5)
    check_images(spec, pts, True)
    osys = oracle_system(spec)
    model = oracle.render(osys, spec.truth.astype(np.float64))
    obs = mocks.Observation(spec, (model + 0.01 * rng.standard_normal(model.shape)).astype(np.float32),
                            (rng.random(model.shape) < 0.8).astype(np.float32) * 1e4, 0.01)
    gsys = gpu_system(spec, obs)
    tp = torch.from_numpy(pts).to(DEV)
    ll = lensed.loglike_batch(tp, np.zeros(len(pts), np.int32), [gsys]).cpu().numpy()
    ref = oracle_loglikes(oracle_system(spec, obs), pts)
    assert np.all(np.abs(ll - ref) <= loglike_tolerance(ref, obs.weight))
    plain = lensed.loglike(tp[0], gsys).cpu().numpy()[0]
    assert abs(plain - ref[0]) <= loglike_tolerance(ref[:1], obs.weight)[0]


def test_mixed_batch_c2_every_point():
    """16 systems of mixed size and subsampling, 512 points each, one graph launch;
    every one of the 8192 log L against the oracle."""
    specs = mocks.c2_specs()
    say("c2 mixed batch, 16 systems x 512 points, all compared")
    gold = golden_file(golden.C2_FILE)
    systems, obs_all, pts_all, sop = [], [], [], []
    for s, spec in enumerate(specs):
        _, obs = observation("c2", s)
        pts = golden.c2_points(spec, s)
        assert str(gold["theta_sha256"][s]) == golden.digest(pts), f"C2 system {s}: points differ"
        assert str(gold["data_sha256"][s]) == golden.digest(obs.data), f"C2 system {s}: mock differs"
        assert str(gold["weight_sha256"][s]) == golden.digest(obs.weight)
        obs_all.append(obs)
        systems.append(gpu_system(spec, obs))
        pts_all.append(pts)
        sop.append(np.full(len(pts), s, np.int32))
    pts = np.concatenate(pts_all)
    sop = np.concatenate(sop)
    ll = lensed.loglike_batch(torch.from_numpy(pts).to(DEV), sop, systems).cpu().numpy()
    worst = 0.0
    for s, spec in enumerate(specs):
        sl = slice(s * 512, (s + 1) * 512)
        ref = gold["loglike"][s]
        ratio = np.abs(ll[sl] - ref) / loglike_tolerance(ref, obs_all[s].weight)
        worst = max(worst, float(ratio.max()))
        bad = np.nonzero(~(ratio <= 1.0))[0]
        assert bad.size == 0, f"{spec.name}: {bad.size} of 512 points off (worst {ratio.max():.3f} x bar)"
    say(f"  worst |delta log L| / bar = {worst:.3f}")


def test_invalid_points_give_nan_only_there():
    spec, obs = observation("c0")
    say("invalid points")
    pts = mocks.points(spec, 6, seed=3)
    pts[1, 1] = 1.5        # q > 1
    pts[3, 13] = -0.2      # R_e < 0
    pts[4, 0] = np.nan
    gsys = gpu_system(spec, obs)
    ll = lensed.loglike_batch(torch.from_numpy(pts).to(DEV), np.zeros(6, np.int32), [gsys]).cpu().numpy()
    assert np.all(np.isnan(ll[[1, 3, 4]]))
    assert np.all(np.isfinite(ll[[0, 2, 5]]))


def test_invalid_arguments_return_status():
    spec, obs = observation("c0")
    gsys = gpu_system(spec, obs)
    tp = torch.from_numpy(spec.truth).to(DEV)
    ctx = lensed.default_context(0)
    from paper_1505_07674_amd import binding
    bad = binding.LensedSystemC.from_buffer_copy(gsys.c_struct)
    out = torch.empty(1, dtype=torch.float64, device=DEV)
    stream = torch.cuda.current_stream().cuda_stream
    import ctypes
    for field, val in [("psf_h", 4), ("nsub", 0), ("nsub", 17), ("height", 0), ("pixscale", -1.0)]:
        b = binding.LensedSystemC.from_buffer_copy(gsys.c_struct)
        setattr(b, field, val)
        rc = binding.lib().lensed_loglike(ctx.handle, ctypes.byref(b), ctypes.c_void_p(tp.data_ptr()),
                                          ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream))
        assert rc == 1, (field, val)
    with pytest.raises(lensed.LensedError):
        lensed.loglike_batch(tp.view(1, 17), [3], [gsys])
    del bad


def test_subsample_on_the_image_of_a_cuspy_source_centre():
    """SIS with theta_E = 0.8 and an n = 4 source centred at (0.2, 0): its centre is
    imaged at x = 1.0 on the axis, exactly where a subsample of the 63x63, N = 3
    grid sits (y = 0 is the middle subsample of the middle row). The float64
    cusp correction must keep the cusp pixel within the bars."""
    say("cusp subsample")
    base = mocks.c1_spec()
    spec = mocks.SystemSpec("cusp_63x63_sub3", 63, 63, 3, mocks.moffat_psf(11, 0.1, 3.0), base.truth,
                            base.prior, np.ones((63, 63), bool), 5, False)
    t = np.array([0.8, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 1.0, 1.0, 0.0,
                  0.2, 0.0, 1.0, 0.05, 4.0, 0.8, 0.3], np.float32)
    t2 = t.copy(); t2[1], t2[2], t2[14] = 0.7, 0.4, 3.0     # elliptical lens, same source
    check_images(spec, np.stack([t, t2]), True)
    check_images(spec, np.stack([t, t2]), False)


@pytest.mark.parametrize("q", [1.0, 0.95, 0.866, 0.8, 0.5, 0.45, 0.2])
def test_every_sie_branch_with_a_subsample_on_the_lens_centre(q):
    """Axis ratios across the four SIE evaluation branches (sphere; polynomials
    for q' <= 1/2; half-angle atan with log atanh for q >= 1/2 and for q < 1/2),
    on a 41x41 grid centred on the lens with N = 3, so that one subsample sits
    exactly on the lens centre (deflection 0 there). Zero lens light and a
    negative source amplitude check the per-pixel amplitudes."""
    say(f"SIE branch q={q}")
    rng = np.random.default_rng(int(q * 1000))
    spec = _custom_spec(41, 41, 3, mocks.gaussian_psf(7, 0.15, 0.06), pixscale=0.06, center=(0.0, 0.0))
    pts = mocks.points(spec, 3, seed=int(q * 100))
    pts[:, 1] = q
    pts[1, 5] = 0.0           # no lens light
    pts[2, 12] = -pts[2, 12]  # negative source amplitude
    check_images(spec, pts, False)
    check_images(spec, pts, True)
