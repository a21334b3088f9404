"""Throughput of the batched forward-lensing log-likelihood on one MI355X.

A step is one batched evaluation of the whole hot path (per-point prologue,
subsample ray-tracing render, PSF + chi^2, float64 finalise) for 4096 parameter
points of the 200x200, 4x4-subsampled, 21x21-Moffat SIE + shear + Sersic model,
with every input resident in HBM. Prints ONE JSON line (rank 0).

Also reported: the plain one-point-per-launch form on the same points, the
roofline of the dominant kernel (render) from per-stage hipEvents, and the FP64
oracle timed on the host cores on a bounded sample.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work per unit (add, mul, fma, div, sqrt and each elementary
# function counted as one op): 84 per subsample of the model, 2 per PSF tap and
# 5 per pixel for the chi^2.
OPS_PER_SUBSAMPLE = 84
# The gradient kernel's per-subsample work, counted the same way: the value and
# the derivatives through both Sersics, the source frame, the lens equation and
# the SIE (q' > 1/2 branch), and the 17 moments they feed (per-point constants
# and the per-point map from moments to partials not counted).
GRAD_OPS_PER_SUBSAMPLE = 159
FP32_PEAK_TFLOPS = 157.3


def box_any(mask, p, q):
    """Pixels within the (2p+1) x (2q+1) box of a True pixel of mask (clipped to the image)."""
    H, W = mask.shape
    c = np.zeros((H + 1, W + 1), np.int64)
    c[1:, 1:] = np.cumsum(np.cumsum(mask.astype(np.int64), 0), 1)
    r0 = np.clip(np.arange(H) - p, 0, H)
    r1 = np.clip(np.arange(H) + p + 1, 0, H)
    c0 = np.clip(np.arange(W) - q, 0, W)
    c1 = np.clip(np.arange(W) + q + 1, 0, W)
    tot = c[r1][:, c1] - c[r0][:, c1] - c[r1][:, c0] + c[r0][:, c0]
    return tot > 0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=4096)
    ap.add_argument("--plain-points", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-points-per-core", type=int, default=10)
    ap.add_argument("--no-mixed", action="store_true", help="skip the 16-system mixed batch line")
    ap.add_argument("--no-next", action="store_true", help="skip the g3k7 and general-model lines")
    ap.add_argument("--grad-points", type=int, default=1024)
    ap.add_argument("--grad-steps", type=int, default=5)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before timing, copy a MIB-MiB device buffer once (a plain copy of known size that scales "
                         "hardware byte counters taken over the same run)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(spec, thetas, per_core):
    """FP64 oracle log L on the host cores: one serial point per thread."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_1505_07674_amd import mocks

    px = float(np.float32(spec.pixscale))
    osys = oracle.System(spec.height, spec.width, px, spec.nsub, spec.psf.astype(np.float64))
    obs = mocks.make_observation(spec, lambda t: oracle.render(osys, np.asarray(t, np.float64)))
    osys = oracle.System(spec.height, spec.width, px, spec.nsub, spec.psf.astype(np.float64),
                         obs.data.astype(np.float64), obs.weight.astype(np.float64))
    cores = min(len(os.sched_getaffinity(0)), 16)
    n = cores * per_core
    sample = [np.asarray(t, np.float64) for t in thetas[:n]]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        vals = list(ex.map(lambda t: oracle.loglike(osys, t), sample))
    dt = time.perf_counter() - t0
    assert all(math.isfinite(v) for v in vals)
    n1 = max(per_core, 4)
    t1 = time.perf_counter()
    for t in sample[:n1]:
        oracle.loglike(osys, t)
    dt1 = time.perf_counter() - t1
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n / dt, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} points of the same 4096-point C1 workload, {per_core} per thread, "
                      f"{dt:.1f} s wall ({cores * dt:.0f} thread-s)",
            "one_core": {"value": n1 / dt1, "unit": "evals/s", "points": n1},
            "cpu_model": cpu}


RENDER_SOURCES = ("internal.h", "sb_device.h", "sie_poly.h", "gk_rules.h", "render.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_c1_batch4096_traffic.json")


def render_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for name in RENDER_SOURCES:
        with open(os.path.join(ROOT, "paper_1505_07674_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per render launch from the committed hardware-counter summary,
    or None when there is none or the render sources changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("sources_sha256") != render_sources_digest():
        return None
    return rec.get("bytes_per_launch")


def mixed_batch(lensed, mocks, dev, stream, c1_ms_per_subsample, steps=5):
    """16 systems of mixed size (64..300 px) and subsampling (N = 2..8), 512 points
    each, in one graph launch: evals/s, subsample-evals/s, and the render stage's
    time per subsample relative to the uniform 200x200 batch (1 = no imbalance cost)."""
    import torch
    specs = mocks.c2_specs()
    systems, thetas, sop = [], [], []
    for s_i, sp in enumerate(specs):
        psf = torch.from_numpy(sp.psf).to(dev)
        rs = lensed.System(psf, pixscale=sp.pixscale, nsub=sp.nsub, height=sp.height, width=sp.width)
        ob = mocks.make_observation(
            sp, lambda t: lensed.render(torch.from_numpy(np.asarray(t, np.float32)).to(dev), rs).cpu().numpy())
        systems.append(lensed.System(psf, torch.from_numpy(ob.data).to(dev), torch.from_numpy(ob.weight).to(dev),
                                     pixscale=sp.pixscale, nsub=sp.nsub))
        thetas.append(mocks.points(sp, 512, seed=mocks.C2_BASE_SEED + 100 + s_i))
        sop += [s_i] * 512
    th = torch.from_numpy(np.concatenate(thetas)).to(dev)
    sop = np.asarray(sop, np.int32)
    out = torch.empty(len(sop), dtype=torch.float64, device=dev)
    ctx = lensed.Context(0)
    log(f"mixed batch: {len(specs)} systems, {len(sop)} points")
    lensed.loglike_batch(th, sop, systems, out=out, ctx=ctx)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        lensed.loglike_batch(th, sop, systems, out=out, ctx=ctx)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    schedule = ctx.batch_schedule()
    ctx.set_profiling(True)
    ctx.stage_times()
    lensed.loglike_batch(th, sop, systems, out=out, ctx=ctx)
    stages, calls = ctx.stage_times()
    ctx.set_profiling(False)
    subs = sum(sp.height * sp.width * sp.nsub ** 2 * 512 for sp in specs)
    assert torch.isfinite(out).all().item()
    return {"value": len(sop) / (ms / 1e3), "unit": "evals/s", "points": len(sop), "systems": len(specs),
            "subsamples_per_launch": subs, "subsample_evals_per_s": subs / (ms / 1e3),
            "render_ms": stages["render"] / calls, "psf_chi2_ms": stages["psf_chi2"] / calls,
            "render_time_per_subsample_vs_uniform": (stages["render"] / calls) / subs / c1_ms_per_subsample,
            "shapes": [f"{sp.height}x{sp.width} N={sp.nsub}" for sp in specs], "schedule": schedule}


# Work per subsample of the 41-parameter general model (two SIEs, shear, four
# Sersics), counted as above: 28 per SIE, 8 for the shear, 2 for beta, 21 per
# Sersic, 2 for the coordinates and 2 to accumulate.
GENERAL41_OPS_PER_SUBSAMPLE = 2 * 28 + 8 + 2 + 4 * 21 + 2 + 2
FP64_PEAK_TFLOPS = 78.6


def next_rows(lensed, mocks, dev, stream, spec, obs, steps=3):
    """Throughput of two extensions on the 200x200 grid: the paper's default
    Gauss-Kronrod rule g3k7 (49 nodes per pixel, float32 like the midpoint
    path) and the 41-parameter general model (float64 render), with its
    gradient."""
    import torch
    out = {}
    psf = torch.from_numpy(spec.psf).to(dev)
    data, weight = torch.from_numpy(obs.data).to(dev), torch.from_numpy(obs.weight).to(dev)

    def timed(call, n_points, ctx):
        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ctx.set_profiling(True)
        ctx.stage_times()
        call()
        st, calls = ctx.stage_times()
        ctx.set_profiling(False)
        return ms, {k: v / calls for k, v in st.items()}

    # g3k7 on the C1 batch
    P = 1024
    ctx = lensed.Context(0)
    gk = lensed.System(psf, data, weight, pixscale=spec.pixscale, nsub=spec.nsub, rule="g3k7")
    th = torch.from_numpy(mocks.points(spec, P, seed=mocks.C1_POINT_SEED)).to(dev)
    sop = np.zeros(P, np.int32)
    res = torch.empty(P, dtype=torch.float64, device=dev)
    log(f"g3k7: {P} points")
    ms, st = timed(lambda: lensed.loglike_batch(th, sop, [gk], out=res, ctx=ctx), P, ctx)
    assert torch.isfinite(res).all().item()
    subs = spec.height * spec.width * 49 * P
    ach = OPS_PER_SUBSAMPLE * subs / (st["render"] * 1e-3) / 1e12
    out["g3k7"] = {"value": P / (ms / 1e3), "unit": "evals/s", "points": P, "nodes_per_pixel": 49,
                   "stage_ms_per_step": st,
                   "roofline": {"bound": "alu", "achieved": ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                "frac": ach / FP32_PEAK_TFLOPS, "kernel": "render",
                                "ops_per_subsample": OPS_PER_SUBSAMPLE, "subsamples_per_launch": subs}}
    ctx.close()

    # the 41-parameter general model (two SIEs, shear, four Sersics, sky), float64 render
    P = 256
    ctx = lensed.Context(0)
    model = lensed.Model(2, mocks.GENERAL_41_PLANES, shear=True, sky=True)
    gs = lensed.System(psf, data, weight, pixscale=spec.pixscale, nsub=spec.nsub)
    th = torch.from_numpy(mocks.general_model_points(P, seed=41)).to(dev)
    sop = np.zeros(P, np.int32)
    res = torch.empty(P, dtype=torch.float64, device=dev)
    log(f"general model (41 parameters): {P} points")
    ms, st = timed(lambda: lensed.loglike_model_batch(th, sop, [gs], model, out=res, ctx=ctx), P, ctx)
    assert torch.isfinite(res).all().item()
    subs = spec.height * spec.width * spec.nsub ** 2 * P
    ach = GENERAL41_OPS_PER_SUBSAMPLE * subs / (st["render"] * 1e-3) / 1e12
    out["general_model_41"] = {"value": P / (ms / 1e3), "unit": "evals/s", "points": P, "params": 41,
                               "stage_ms_per_step": st,
                               "roofline": {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
                                            "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
                                            "kernel": "model_render (float64 rays, float32 profile fractions)",
                                            "ops_per_subsample": GENERAL41_OPS_PER_SUBSAMPLE,
                                            "subsamples_per_launch": subs}}
    # and its adjoint (one component per pass, float64 dual numbers)
    P = 64
    th = th[:P].contiguous()
    log(f"general model (41 parameters) gradients: {P} points")
    ms, st = timed(lambda: lensed.loglike_model_grad(th, gs, model, ctx=ctx), P, ctx)
    out["general_model_41_grad"] = {"value": P / (ms / 1e3), "unit": "gradients/s", "points": P, "params": 41,
                                    "passes": 2 + 4 + 1, "stage_ms_per_step": st}
    ctx.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by points across GPUs; this benchmark runs one GPU's share)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1505_07674_amd as lensed
    from paper_1505_07674_amd import mocks

    dev = torch.device("cuda:0")
    spec = mocks.c1_spec()
    psf = torch.from_numpy(spec.psf).to(dev)
    rsys = lensed.System(psf, pixscale=spec.pixscale, nsub=spec.nsub, height=spec.height, width=spec.width)
    # synthetic mock rendered by the library itself (inputs only; no parity claim here)
    obs = mocks.make_observation(
        spec, lambda t: lensed.render(torch.from_numpy(np.asarray(t, np.float32)).to(dev), rsys).cpu().numpy())
    gsys = lensed.System(psf, torch.from_numpy(obs.data).to(dev), torch.from_numpy(obs.weight).to(dev),
                         pixscale=spec.pixscale, nsub=spec.nsub)
    P = args.points
    pts = mocks.points(spec, P, seed=mocks.C1_POINT_SEED)
    theta = torch.from_numpy(pts).to(dev)
    sop = np.zeros(P, np.int32)
    out = torch.empty(P, dtype=torch.float64, device=dev)
    ctx = lensed.default_context(0)
    stream = torch.cuda.current_stream()

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)      # one elementwise kernel: n floats read, n written
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + {args.copy_calibration} MiB written "
            "by one elementwise kernel")
        del src, dst

    log(f"batched: {P} points, warmup {args.warmup}")
    for _ in range(args.warmup):
        lensed.loglike_batch(theta, sop, [gsys], out=out, ctx=ctx)
    torch.cuda.synchronize()
    log(f"batched: timing {args.steps} steps")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        lensed.loglike_batch(theta, sop, [gsys], out=out, ctx=ctx)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    value = P * args.steps / (ms_total / 1e3)
    assert torch.isfinite(out).all().item(), "non-finite log L in the timed batch"
    schedule = ctx.batch_schedule()
    rendered = ctx.batch_rendered()
    assert rendered["subsamples"] == spec.height * spec.width * spec.nsub ** 2 * P

    # per-stage kernel durations over an equal number of profiled steps
    log("batched: per-stage hipEvent timing")
    ctx.set_profiling(True)
    ctx.stage_times()
    for _ in range(args.steps):
        lensed.loglike_batch(theta, sop, [gsys], out=out, ctx=ctx)
    stages, calls = ctx.stage_times()
    ctx.set_profiling(False)
    stage_ms = {k: v / calls for k, v in stages.items()}
    subs = spec.height * spec.width * spec.nsub ** 2
    render_flops = OPS_PER_SUBSAMPLE * subs * P
    achieved = render_flops / (stage_ms["render"] * 1e-3) / 1e12
    taps = spec.psf.shape[0] * spec.psf.shape[1]
    psf_flops = (2 * taps + 5) * spec.height * spec.width * P
    psf_tflops = psf_flops / (stage_ms["psf_chi2"] * 1e-3) / 1e12

    # plain form: one launch sequence per point, back-to-back, one sync at the end
    n_plain = min(args.plain_points, P)
    log(f"plain: {n_plain} points")
    outs = torch.empty(n_plain, dtype=torch.float64, device=dev)
    for i in range(min(8, n_plain)):
        lensed.loglike(theta[i], gsys, out=outs[i:i + 1], ctx=ctx)
    torch.cuda.synchronize()
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    for i in range(n_plain):
        lensed.loglike(theta[i], gsys, out=outs[i:i + 1], ctx=ctx)
    p1.record(stream)
    torch.cuda.synchronize()
    plain_value = n_plain / (p0.elapsed_time(p1) / 1e3)
    rel = (outs - out[:n_plain]).abs() / out[:n_plain].abs().clamp_min(1.0)
    assert rel.max().item() < 1e-5, "plain and batched log L disagree"
    # plain with a host sync per point, as a sampler calling one point at a time would
    n_sync = min(256, n_plain)
    ts = time.perf_counter()
    for i in range(n_sync):
        lensed.loglike(theta[i], gsys, out=outs[i:i + 1], ctx=ctx)
        outs[i].item()
    plain_sync_value = n_sync / (time.perf_counter() - ts)

    # adjoint: log L and its 17-gradient for the C3 configuration
    G = args.grad_points
    log(f"gradient: {G} points, {args.grad_steps} steps")
    gpts = torch.from_numpy(mocks.points(spec, G, seed=mocks.C3_SEED)).to(dev)
    lensed.loglike_grad(gpts, gsys, ctx=ctx)
    torch.cuda.synchronize()
    g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    g0.record(stream)
    for _ in range(args.grad_steps):
        gll, gg = lensed.loglike_grad(gpts, gsys, ctx=ctx)
    g1.record(stream)
    torch.cuda.synchronize()
    grad_value = G * args.grad_steps / (g0.elapsed_time(g1) / 1e3)
    assert torch.isfinite(gg).all().item()
    # the gradient kernel alone: stage events over profiled passes of the same launch
    ctx.set_profiling(True)
    ctx.stage_times()
    for _ in range(args.grad_steps):
        lensed.loglike_grad(gpts, gsys, ctx=ctx)
    gstages, gcalls = ctx.stage_times()
    ctx.set_profiling(False)
    grad_stage_ms = {k: v / gcalls for k, v in gstages.items()}
    # it evaluates only pixels that A^T rho reaches: the w > 0 support dilated by the PSF box
    ph, pw = spec.psf.shape
    vis_px = int(box_any(obs.weight > 0, ph // 2, pw // 2).sum())
    grad_subs = vis_px * spec.nsub ** 2 * G
    grad_achieved = GRAD_OPS_PER_SUBSAMPLE * grad_subs / (grad_stage_ms["grad"] * 1e-3) / 1e12

    # masked form: only the pixels the chi^2 can see (same log L, bit for bit)
    log("masked: same batch, visible pixels only")
    out_m = torch.empty_like(out)
    lensed.loglike_batch(theta, sop, [gsys], out=out_m, ctx=ctx, masked=True)
    torch.cuda.synchronize()
    vis = ctx.batch_rendered()
    m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    m0.record(stream)
    for _ in range(args.steps):
        lensed.loglike_batch(theta, sop, [gsys], out=out_m, ctx=ctx, masked=True)
    m1.record(stream)
    torch.cuda.synchronize()
    masked_ms = m0.elapsed_time(m1) / args.steps
    assert torch.equal(out_m, out), "masked and all-pixel log L differ"
    masked = {"value": P / (masked_ms / 1e3), "unit": "evals/s", "points": P, "ms_per_step": masked_ms,
              "rendered_pixel_fraction": vis["pixels"] / rendered["pixels"],
              "form": "only the pixels within the PSF footprint of w > 0 rendered, only PSF tiles with w > 0 "
                      "convolved; log L identical bit for bit to the all-pixel batch"}

    extensions = None if args.no_next else next_rows(lensed, mocks, dev, stream, spec, obs)

    mixed = None
    if not args.no_mixed:
        mixed = mixed_batch(lensed, mocks, dev, stream, stage_ms["render"] / (subs * P))

    result = {
        "metric": "log-likelihood evals/sec at 200x200, 4x4 subsample (batched)",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "c1_200x200_sie_shear_sersic_sub4_moffat21_batch4096",
                   "points_per_step": P, "image": [spec.height, spec.width], "nsub": spec.nsub,
                   "psf": "21x21 Moffat beta=3 FWHM 0.1 arcsec", "params": 17,
                   "mask": "annulus 0.3-3.0 arcsec (all pixels rendered)"},
        "plain": {"value": plain_value, "unit": "evals/s", "points": n_plain,
                  "form": "one prologue/render/psf/finalize launch sequence per point, one sync"},
        "plain_host_sync": {"value": plain_sync_value, "unit": "evals/s", "points": n_sync,
                            "form": "one point per call, host sync after each (not used for the ratio)"},
        "batched_over_plain": value / plain_value,
        "adjoint": {"value": grad_value, "unit": "gradients/s", "points": G,
                    "form": "log L and d log L/d theta (17) per point, one graph launch per step",
                    "stage_ms_per_step": grad_stage_ms,
                    "roofline": {"bound": "alu", "achieved": grad_achieved, "peak": FP32_PEAK_TFLOPS,
                                 "unit": "TFLOP/s", "frac": grad_achieved / FP32_PEAK_TFLOPS, "kernel": "grad",
                                 "ops_per_subsample": GRAD_OPS_PER_SUBSAMPLE, "subsamples_per_launch": grad_subs,
                                 "pixels_per_point": vis_px}},
        "stage_ms_per_step": stage_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": measured_traffic(),
                     "kernel": "render", "ops_per_subsample": OPS_PER_SUBSAMPLE,
                     "subsamples_per_launch": subs * P},
        "psf_chi2_tflops": psf_tflops,
        "schedule": {"psf_tile": schedule["psf_tile"], "render_pixels_per_thread": schedule["render_pixels_per_thread"],
                     "render_block": schedule["render_block"],
                     "chosen_by": ("fixed by LENSED_RENDER_PPT / LENSED_RENDER_BLOCK"
                                   if os.environ.get("LENSED_RENDER_PPT") or os.environ.get("LENSED_RENDER_BLOCK")
                                   else "autotuner (timed on this launch)")},
        "masked": masked,
        "mixed_batch": mixed,
        "extensions": extensions,
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on host cores")
        result["cpu_baseline"] = cpu_baseline(spec, pts, args.cpu_points_per_core)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
