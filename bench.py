"""Throughput of PSF-matched difference imaging on one MI355X.

One step is the whole path over one synthetic full IMX455 frame pair
(9576 x 6388 uint16): calibrate the 5 reference frames and coadd them with a
3-sigma clip (one fused kernel), calibrate the science frame, fit the spatially varying kernel
(21x21, 31 Gaussian bases, degree-2 polynomial, 16x16 sub-tile partials,
192 unknowns), expand it, convolve-subtract, and detect.  Inputs (raw frames
and calibration masters) are resident in HBM before the timed region.

Prints ONE JSON line with the metric, the roofline of the dominant kernel
(per-kernel device times from HIP events on the launch stream) and the FP64
CPU oracle timed on a bounded crop of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP32_VALU_TFLOPS = 78.6       # one FP32 op per lane per clock (packed FP32 disabled)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--width", type=int, default=9576)
    p.add_argument("--height", type=int, default=6388)
    p.add_argument("--stars", type=int, default=60000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--two-cameras", type=int, default=0,
                   help="also time two cameras' steps on two streams (its launches overlap, "
                        "so a kernel trace of such a run mixes concurrent kernels)")
    p.add_argument("--cpu-crop", type=int, default=1024)
    p.add_argument("--batch-frames", type=int, default=20)
    p.add_argument("--batch-cutouts", type=int, default=4000)
    p.add_argument("--batch-steps", type=int, default=3)
    p.add_argument("--sur-frames", type=int, default=400)
    p.add_argument("--sur-epochs", type=int, default=15)
    p.add_argument("--copy-probe", action="store_true",
                   help="only run a plain 1 GiB device copy (5 times), the reference for "
                        "scaling hardware byte counters")
    return p.parse_args()


def copy_probe():
    """A plain elementwise copy kernel over 1 GiB (y = x * 1), five times: each
    dispatch reads and writes exactly 2^30 bytes, so FETCH_SIZE / WRITE_SIZE
    counters of these dispatches give the scale from counter units to bytes.
    (An elementwise kernel rather than copy_, which may go to a DMA engine
    that per-dispatch counters do not see.)"""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        torch.mul(x, 1.0, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    print(json.dumps({"copy_bytes": 1 << 30, "ms": round(ms, 4),
                      "GB/s_read+write": round(2 * (1 << 30) / ms / 1e6, 1)}), flush=True)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Sources that decide the frame fit's memory traffic (kernel and its launch).
FIT_SOURCES = ["paper_2207_14304_amd/csrc/fit_accum8.h", "paper_2207_14304_amd/csrc/fit_accum.h",
               "paper_2207_14304_amd/csrc/k_fit_fp32.hip", "paper_2207_14304_amd/csrc/k_fit.hip"]
TRAFFIC_FILE = "profiles/fit_accum_traffic.md"


def fit_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in FIT_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the frame fit from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by the same
    counter on a plain 1 GiB copy kernel), or None when the kernel sources
    have changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
    if kv.get("source_sha256") != fit_source_hash():
        return None
    try:
        return int(float(kv["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def algorithmic_work(name, spec, npix, n_ref):
    """(kind, amount per launch) of the algorithmic work of an internal kernel."""
    D = spec.spatial_degree
    K = 2 * spec.half_width + 1
    if name == "calibrate":
        return "hbm", 20.0 * npix                    # u16 + 2 f32 + u8 in, 2 f32 + u8 out
    if name == "coadd":
        return "hbm", (9.0 * n_ref + 10.0) * npix    # n x (2 f32 + u8) in, 2 f32 + 2 u8 out
    if name == "calibrate_coadd":
        return "hbm", (2.0 * n_ref + 19.0) * npix    # n u16 + 2 f32 + u8 in, 2 f32 + 2 u8 out
    if name == "detect_map":
        return "hbm", 14.0 * npix                    # 2 f32 + u8 in, f32 + u8 out
    if name == "subtract":
        # per tap and pixel: kernel evaluation (D=2: 2 FMA), model FMA, variance MUL + FMA
        per_tap = {0: 4.0, 1: 7.0, 2: 9.0}[D]
        return "alu", per_tap * K * K * npix
    if name == "fit_accum":
        # symmetric 32x32 moments for each of the 2D+1 x-powers (FMA = 2 flop)
        return "mfma", (2 * D + 1) * 528 * 2.0 * npix
    return None, 0.0


def cpu_baseline(fp, crop, spec_o):
    """FP64 oracle on a crop x crop window of the same frames (whole path)."""
    import oracle
    from paper_2207_14304_amd import synth
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] + [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    y0 = (fp.H - crop) // 2
    x0 = (fp.W - crop) // 2
    sl = (slice(y0, y0 + crop), slice(x0, x0 + crop))
    t0 = time.perf_counter()
    refs = [oracle.calibrate(r[sl], fp.dark[sl], fp.flat[sl], fp.bpm[sl]) for r in fp.ref_raw]
    ref, rv, rm, _ = oracle.coadd([r[0] for r in refs], [r[1] for r in refs],
                                  [r[2] for r in refs], 3.0, 5)
    cs, vs, ms = oracle.calibrate(fp.sci_raw[sl], fp.dark[sl], fp.flat[sl], fp.bpm[sl])
    co, st, nf = oracle.fit_kernel(ref, rv, rm, cs, vs, ms, spec_o)
    stamps, bg = oracle.expand_kernel(co, spec_o)
    D, V, dm, _, _ = oracle.subtract(stamps, bg, ref, rv, rm, cs, vs, ms, spec_o)
    oracle.detect(D, V, dm, 5.0, synth.psf_image(7, 2.6))
    dt = time.perf_counter() - t0
    return {"value": round(crop * crop / dt / 1e6, 4), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle",
            "sample": f"whole path (5-frame coadd, D=2 h=10 fit, subtract, detect) on the "
                      f"central {crop}x{crop} crop of the same frames, {dt:.1f} s"}


def batch_leg(args, torch, argus, synth):
    """Cutout batching: many cameras' frames, one persistent graph launch."""
    from paper_2207_14304_amd import synth_torch
    W, H, nf = args.width, args.height, args.batch_frames
    t0 = time.perf_counter()
    ctx = argus.Context(0)
    dark = torch.zeros((H, W), dtype=torch.float32, device="cuda")
    flat = torch.ones((H, W), dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(40)
    frames, fr, xs0, ys0, Ls = [], [], [], [], []
    for f in range(nf):
        fwhm = float(rng.uniform(1.5, 4.0))
        sci_raw, ref_raw, sx, sy = synth_torch.make_pair(W, H, args.stars, 40 + f, fwhm)
        planes = []
        for raw in (ref_raw, sci_raw):
            c = torch.empty((H, W), dtype=torch.float32, device="cuda")
            v = torch.empty_like(c)
            m = torch.empty((H, W), dtype=torch.uint8, device="cuda")
            ctx.calibrate(raw, dark, flat, None, 1.0, 1.7, 65535, c, v, m)
            planes += [c, v, m]
        del sci_raw, ref_raw
        frames.append(tuple(planes))
        a, b, L = synth.draw_cutouts(40 + f, W, H, sx, sy, args.batch_cutouts)
        fr += [f] * len(a)
        xs0 += list(a)
        ys0 += list(b)
        Ls += list(L)
    torch.cuda.synchronize()
    log(f"batch: {nf} frame pairs generated and calibrated in {time.perf_counter() - t0:.1f} s")
    # FP64 row moments: the small cutouts' systems need them for the
    # 1e-4 sigma difference bar
    spec = argus.make_spec(half_width=7, precision=argus.FP64)
    b = argus.Batch(ctx, spec, fr, xs0, ys0, Ls, [W] * nf, [H] * nf)
    n = b.n
    outs = [torch.empty(b.arena, dtype=torch.float32, device="cuda"),
            torch.empty(b.arena, dtype=torch.float32, device="cuda"),
            torch.empty(b.arena, dtype=torch.uint8, device="cuda"),
            torch.empty(b.arena, dtype=torch.uint8, device="cuda"),
            torch.empty((n, 32), dtype=torch.float64, device="cuda"),
            torch.empty(n, dtype=torch.float64, device="cuda"),
            torch.empty(n, dtype=torch.int64, device="cuda"),
            torch.empty(n, dtype=torch.int32, device="cuda"),
            torch.empty(n, dtype=torch.int32, device="cuda")]
    t1 = time.perf_counter()
    ctx.batch_run(b, frames, 5.0, *outs)          # autotune + graph capture + run
    torch.cuda.synchronize()
    log(f"batch: first run (autotune over candidates) {time.perf_counter() - t1:.1f} s, "
        f"choice {b.info()}")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.batch_steps):
        ctx.batch_run(b, frames, 5.0, *outs)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.batch_steps
    gpix = float(np.sum(np.asarray(Ls, np.float64) ** 2)) / 1e9
    st = outs[7].cpu().numpy()
    choice, tuned_ms, ncand = b.info()
    res = {"value": round(gpix * 1e6 / ms, 2), "unit": "Mpix/s", "ms": round(ms, 3),
           "cutouts": n, "frames": nf, "cutout_gpix": round(gpix, 4),
           "side_px": [int(min(Ls)), int(max(Ls))], "solves_ok": int((st == 0).sum()),
           "autotune": {"choice": choice, "candidates": ncand, "best_ms": round(tuned_ms, 3)},
           "workload": f"{nf} cameras x {args.batch_cutouts} cutouts, sides log-uniform 64-512, "
                       f"constant 15x15 kernel each (FP64 row moments), one graph launch"}
    log("batch: " + json.dumps(res))
    b.close()
    del frames, outs
    torch.cuda.empty_cache()
    return res


def surrogate_leg(args, torch, argus):
    """Learned kernel surrogate: GPU training throughput, then per-frame plain
    PER_TILE path vs surrogate path on 1024^2 frames (4x4 tiles, 15x15
    kernel), acceptance and kernel error against the noise-free fit."""
    from paper_2207_14304_amd import surrogate as sur
    ctx = argus.Context(0)
    t0 = time.perf_counter()
    X, V, T = sur.build_training_set(ctx, args.sur_frames, 1, n_stars=(3000, 20000), log=log)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    Ts, mu, sd = sur.standardize(T)
    cnn = argus.CNN(ctx, max_tiles=64)
    cnn.set_weights(sur.init_weights(1))
    n = X.shape[0]
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    steps = 0
    for ep in range(args.sur_epochs):
        lr = 2e-3 if ep < 0.7 * args.sur_epochs else 4e-4
        steps += len(sur.train(cnn, X, V, Ts, 1, 32, lr, seed=100 + ep))
        log(f"surrogate: epoch {ep} queued ({n} samples)")
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1)
    samples_s = steps * 32 / (train_ms / 1e3)
    # 3 x 1.74 GMAC per training sample (forward, data and weight gradients)
    train_tflops = samples_s * 3 * 1.74e9 * 2 / 1e12
    cnn.set_weights(sur.fold_standardization(cnn.get_weights(), mu.cpu().numpy(),
                                             sd.cpu().numpy()))
    del X, V, T, Ts
    # inference on configuration-1 frames (1024^2, 3000 stars, FWHM 2.0/2.6)
    W = H = 1024
    sp = sur.spec()
    path = sur.SurrogatePath(ctx, cnn, W, H)
    cond = sur.Conditions(2.0, 2.6, 0.0, 0.0, 800.0, 1.05)
    frames = [sur.Frame(ctx, W, H, 3000, 9000 + i, cond, noise_free=True) for i in range(4)]
    B = sur.basis_stamps(ctx)
    rows = sur.evaluate(ctx, path, frames, B)

    def timed(fn, reps=5):
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            for fr in frames:
                fn(fr)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / (reps * len(frames))

    def plain(fr):
        sur.TileFits(ctx, fr.planes, sp)

    def surrogate_only(fr):
        path.predict(fr.planes)
        path.select(None, ref_chi2_dof=1.0)
        path.subtract_final(fr.planes)

    def evaluation_mode(fr):
        tf = sur.TileFits(ctx, fr.planes, sp)
        path.predict(fr.planes)
        path.select(tf)
        path.subtract_final(fr.planes)

    ms_plain = timed(plain)
    ms_sur = timed(surrogate_only)
    ms_eval = timed(evaluation_mode)
    ok = [r for r in rows if r["status"] == 0]
    med = lambda k: float(np.nanmedian([r[k] for r in ok]))
    res = {"train": {"samples": n, "frames": args.sur_frames, "epochs": args.sur_epochs,
                     "generate_s": round(t_gen, 2), "samples_per_s": round(samples_s, 1),
                     "TFLOP/s_bf16": round(train_tflops, 1),
                     "frac_bf16_peak": round(train_tflops / 2500.0, 4)},
           "plain_per_tile_mpix_s": round(W * H / (ms_plain / 1e3) / 1e6, 1),
           "surrogate_path_mpix_s": round(W * H / (ms_sur / 1e3) / 1e6, 1),
           "both_fits_mpix_s": round(W * H / (ms_eval / 1e3) / 1e6, 1),
           "acceptance": round(float(np.mean([r["accepted"] for r in ok])), 3),
           "final_over_plain_chi2dof_max": round(max(r["chi2dof_final"] / r["chi2dof_plain"]
                                                     for r in ok), 5),
           "kernel_err_vs_noise_free": {"plain": round(med("err_plain"), 4),
                                        "surrogate": round(med("err_sur"), 4)},
           "model_err_vs_noise_free": {"plain": round(med("model_err_plain"), 4),
                                       "surrogate": round(med("model_err_sur"), 4)},
           "workload": f"train: {args.sur_frames} 1024^2 pairs (seeing 1.5-4.0, ell 0-0.2, sky "
                       f"200-3000), noise-free plain-fit targets, {args.sur_epochs} epochs, batch "
                       f"32 tiles; infer: 4 configuration-1 frames, 4x4 tiles, 15x15 kernel"}
    log("surrogate: " + json.dumps(res))
    cnn.close()
    return res


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_2207_14304_amd import argus, synth
    from paper_2207_14304_amd.pipeline import Pipeline

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(2)
    W, H = args.width, args.height
    t0 = time.perf_counter()
    fp = synth.make_pair(W, H, args.stars, 2, None, None, True, 5, True, 800.0, 1.05, 20,
                         cosmic_rate=1e-5)
    log(f"generated {W}x{H} pair in {time.perf_counter() - t0:.1f} s")
    spec = argus.make_spec(sigmas=(0.7, 1.5, 3.0), degrees=(4, 3, 2), half_width=10,
                           spatial_degree=2, bg_degree=2, tiles_x=16, tiles_y=16)
    ctx = argus.Context(0)
    psf = synth.psf_image(7, 2.6)
    pipe = Pipeline(ctx, W, H, spec, psf)
    pipe.set_masters(fp.dark, fp.flat, fp.bpm)

    def up(a):
        return torch.from_numpy(a.view(np.int16)).cuda().view(torch.uint16)

    refs = [up(r) for r in fp.ref_raw]
    sci = up(fp.sci_raw)
    torch.cuda.synchronize()

    def step():
        pipe.build_reference(refs)
        pipe.difference(sci)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i} done; status {pipe.status.cpu().tolist()} cands {int(pipe.n_cands.item())}")
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # per-kernel device times: HIP events around every launch on the launch
    # stream, recorded without synchronisation during the timed steps
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1) / args.steps
    npix = W * H
    log(f"timed {args.steps} steps: {ms:.3f} ms/step (wall {wall:.2f} s)")

    names = ["calibrate", "calibrate_coadd", "fit_accum", "fit_reduce", "fit_solve",
             "subtract", "detect_map"]
    kt = {n: float(ctx.kernel_time_ms(n)) for n in names}     # average over the timed launches
    kt = {n: t for n, t in kt.items() if t >= 0}
    ctx.set_timing(False)
    log("kernel ms: " + json.dumps({k: round(v, 4) for k, v in kt.items()}))
    stages = {}
    for n, t in kt.items():
        kind, work = algorithmic_work(n, spec, npix, 5)
        if kind == "hbm":
            stages[n] = {"ms": round(t, 4), "GB/s": round(work / t / 1e6, 1),
                         "frac_hbm": round(work / t / 1e6 / PEAK_HBM_GBS, 4)}
        elif kind in ("alu", "mfma"):
            peak = PEAK_FP32_VALU_TFLOPS if kind == "alu" else PEAK_FP32_MFMA_TFLOPS
            stages[n] = {"ms": round(t, 4), "TFLOP/s": round(work / t / 1e9, 2),
                         "frac": round(work / t / 1e9 / peak, 4), "bound": kind}
        else:
            stages[n] = {"ms": round(t, 4)}
    dom = max((n for n in kt if algorithmic_work(n, spec, npix, 5)[0]), key=lambda n: kt[n])
    kind, work = algorithmic_work(dom, spec, npix, 5)
    if kind == "hbm":
        ach, peak, unit = work / kt[dom] / 1e6, PEAK_HBM_GBS, "GB/s"
    else:
        ach = work / kt[dom] / 1e9
        peak = PEAK_FP32_VALU_TFLOPS if kind == "alu" else PEAK_FP32_MFMA_TFLOPS
        unit = "TFLOP/s"
    roof = {"bound": kind, "kernel": dom, "achieved": round(ach, 2), "peak": peak, "unit": unit,
            "frac": round(ach / peak, 4),
            "traffic": measured_traffic() if dom == "fit_accum" else None}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        spec_o = oracle.KernelSpec(sigmas=(0.7, 1.5, 3.0), degrees=(4, 3, 2), half_width=10,
                                   spatial_degree=2, bg_degree=2, tiles_x=2, tiles_y=2)
        cpu = cpu_baseline(fp, args.cpu_crop, spec_o)
        log("cpu baseline: " + json.dumps(cpu))

    # per-frame difference with the reference resident (calibrate the science
    # frame, fit, expand, subtract, detect): the per-frame cost once the
    # reference of a pointing is built
    torch.cuda.synchronize()
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record(stream)
    for _ in range(args.steps):
        pipe.difference(sci)
    f1.record(stream)
    torch.cuda.synchronize()
    ms_frame = f0.elapsed_time(f1) / args.steps
    log(f"per-frame difference: {ms_frame:.3f} ms")

    # precision variants of the fit on the same frame: the fit accumulation
    # time and the chi^2/dof of the subtraction each one gives, against FP32
    prec = {}
    chi = {}
    for name, pv in (("fp32", argus.FP32), ("bf16x3", argus.BF16X3), ("fp64", argus.FP64)):
        pipe.spec = argus.make_spec(sigmas=(0.7, 1.5, 3.0), degrees=(4, 3, 2), half_width=10,
                                    spatial_degree=2, bg_degree=2, tiles_x=16, tiles_y=16,
                                    precision=pv)
        ctx.set_timing(True)
        for _ in range(3):
            pipe.fit()
        t_fit = ctx.kernel_time_ms("fit_accum")
        ctx.set_timing(False)
        pipe.subtract()
        c2 = float(pipe.chi2.sum().item()) / max(float(pipe.n_chi2.sum().item()) - 192, 1.0)
        chi[name] = c2
        prec[name] = {"fit_accum_ms": round(t_fit, 3),
                      "status_ok": bool((pipe.status == 0).all().item())}
    for name in prec:
        prec[name]["chi2dof_over_fp32"] = round(chi[name] / chi["fp32"], 8)
    pipe.spec = spec
    log("precision variants: " + json.dumps(prec))

    # two cameras sharing the GPU: a second pipeline with its own context on
    # its own stream (both streams at the default priority), the two cameras'
    # steps interleaved, so one camera's single-workgroup solve and the tails
    # of its kernels overlap the other's work; aggregate throughput of both
    two = None
    if args.two_cameras:
        ctx2 = argus.Context(0)
        pipe2 = Pipeline(ctx2, W, H, spec, psf)
        pipe2.set_masters(fp.dark, fp.flat, fp.bpm)
        s_a, s_b = torch.cuda.Stream(), torch.cuda.Stream()

        def both(n):
            for _ in range(n):
                with torch.cuda.stream(s_a):
                    step()
                with torch.cuda.stream(s_b):
                    pipe2.build_reference(refs)
                    pipe2.difference(sci)

        torch.cuda.synchronize()
        both(2)
        torch.cuda.synchronize()
        cur = torch.cuda.current_stream()
        t0e, t1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ea, eb = torch.cuda.Event(), torch.cuda.Event()
        t0e.record(cur)
        s_a.wait_event(t0e)
        s_b.wait_event(t0e)
        both(args.steps)
        ea.record(s_a)
        eb.record(s_b)
        cur.wait_event(ea)
        cur.wait_event(eb)
        t1e.record(cur)
        torch.cuda.synchronize()
        ms2 = t0e.elapsed_time(t1e)
        same = bool(torch.equal(pipe.diff, pipe2.diff) and torch.equal(pipe.coeffs, pipe2.coeffs))
        two = {"value": round(2 * args.steps * npix / (ms2 / 1e3) / 1e6, 2), "unit": "Mpix/s",
               "ms_per_frame": round(ms2 / (2 * args.steps), 4), "identical_to_one_camera": same,
               "workload": "two cameras, each a full step (5-frame calibrate + coadd, "
                           "difference), on two streams with interleaved steps"}
        log("two cameras: " + json.dumps(two))
        del pipe2
        ctx2.close()

    del refs, sci, pipe
    torch.cuda.empty_cache()
    variants = {"precision": prec, "per_frame_difference": {
        "value": round(npix / (ms_frame / 1e3) / 1e6, 2), "unit": "Mpix/s",
        "ms": round(ms_frame, 4),
        "workload": "science calibrate + fit + expand + subtract + detect, reference resident"}}
    if two is not None:
        variants["two_cameras"] = two
    if args.batch_frames > 0:
        variants["batch"] = batch_leg(args, torch, argus, synth)
    if args.sur_frames > 0:
        variants["surrogate"] = surrogate_leg(args, torch, argus)

    value = npix / (ms / 1e3) / 1e6
    out = {
        "metric": "Mpix/s PSF-matched difference imaging (61 MP frame)",
        "value": round(value, 2), "unit": "Mpix/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"IMX455 pair {W}x{H} u16, 5-frame clipped reference + science, "
                               f"21x21 kernel, 31 bases, degree-2 spatial, 192 unknowns, "
                               f"16x16 sub-tiles, detect at 5 sigma",
                   "frame_px": npix, "plain_or_surrogate": "plain"},
        "roofline": roof,
        "stages": stages,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
