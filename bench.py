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
FP32_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--points", type=int, default=4096)
    ap.add_argument("--plain-points", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-points-per-core", type=int, default=10)
    ap.add_argument("--no-mixed", action="store_true", help="skip the 16-system mixed batch line")
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
            "shapes": [f"{sp.height}x{sp.width} N={sp.nsub}" for sp in specs]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported by this build "
              "(the path shards by points across GPUs, but no multi-GPU run is part of it)", file=sys.stderr)
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
                    "form": "log L and d log L/d theta (17) per point, one graph launch per step"},
        "stage_ms_per_step": stage_ms,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": measured_traffic(),
                     "kernel": "render", "ops_per_subsample": OPS_PER_SUBSAMPLE,
                     "subsamples_per_launch": subs * P},
        "psf_chi2_tflops": psf_tflops,
        "mixed_batch": mixed,
        "wall_s_timed": wall,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on host cores")
        result["cpu_baseline"] = cpu_baseline(spec, pts, args.cpu_points_per_core)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
