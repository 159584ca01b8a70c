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
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP32_VALU_TFLOPS = 78.6       # one FP32 op per lane per clock (packed FP32 disabled)
PEAK_FP32_PUBLISHED = 157.3        # published FP32 vector peak (packed FP32 ops)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--width", type=int, default=9576)
    p.add_argument("--height", type=int, default=6388)
    p.add_argument("--stars", type=int, default=60000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--two-cameras", type=int, default=0,
                   help="also time two cameras' steps on two streams (its launches overlap, "
                        "so a kernel trace of such a run mixes concurrent kernels)")
    p.add_argument("--cpu-tiles", type=int, default=16,
                   help="sub-tiles (of 16 x 16) the CPU oracle baseline is timed on")
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
TRAFFIC_FILE = "profiles/frame_path_hbm_traffic.md"


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


def _limit_blas_threads():
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(1)
    except Exception:
        pass


def _oracle_tile_fit(task):
    """Pool worker, phase 1: calibrate the 5 reference frames and the science
    frame on a tile plus halo, coadd, and the tile's normal equations (the fit
    set restricted to the tile's own pixels; full-frame coordinates)."""
    import oracle
    raws, sci_raw, dark, flat, bpm, inner, coords, spec_o = task
    refs = [oracle.calibrate(r, dark, flat, bpm) for r in raws]
    ref, rv, rm, _ = oracle.coadd([r[0] for r in refs], [r[1] for r in refs],
                                  [r[2] for r in refs], 3.0, 5)
    cs, vs, ms = oracle.calibrate(sci_raw, dark, flat, bpm)
    (a, b), (c, d) = inner
    fit_ms = np.full(ms.shape, oracle.BAD, np.uint8)       # outside the tile: not fit here
    fit_ms[a:b, c:d] = ms[a:b, c:d]
    A, bb, nf = oracle.normal_equations(ref, rv, rm, cs, vs, fit_ms, spec_o, coords=coords)
    return A.sum(0), bb.sum(0), int(nf.sum()), (ref, rv, rm, cs, vs, ms)


def _oracle_tile_diff(task):
    """Pool worker, phase 2: subtraction with the global kernel and detection
    on a tile plus halo; candidates counted on the tile's own pixels."""
    import oracle
    planes, stamps, bg, inner, coords, spec_o, psf = task
    D, V, dm, _, _ = oracle.subtract(stamps, bg, *planes, spec_o, coords=coords)
    _, _, c = oracle.detect(D, V, dm, 5.0, psf)
    (a, b), (cc, d) = inner
    return int(((c["y"] >= a) & (c["y"] < b) & (c["x"] >= cc) & (c["x"] < d)).sum())


def cpu_baseline(fp, spec_o, n_tiles, tiles=16):
    """FP64 oracle timed on the host cores: a process pool with one worker per
    core (BLAS at one thread each) over a sample of the frame's 16 x 16
    sub-tiles, each read with a halo (the kernel half-width plus the PSF
    half-width): per tile calibration of the five reference frames and the
    science frame, coadd and normal equations; one FP64 solve of their sum;
    per tile subtraction and detection.  Mpix/s = sampled tile pixels / wall
    time.  Also the whole path on the 1024^2 CPU-sized pair in one process
    on one core.  At most 16 workers (the host cores that go with one GPU)."""
    import multiprocessing as mp
    import oracle
    from paper_2207_14304_amd import synth
    cores = min(len(os.sched_getaffinity(0)), 16)     # the GPU's share of the host
    W, H = fp.W, fp.H
    h, r = spec_o.half_width, 7
    halo = h + r
    xt, yt = oracle.norm_coords(W, H)
    psf = synth.psf_image(r, 2.6)
    rng = np.random.default_rng(0)
    pick = sorted(rng.choice(tiles * tiles, size=min(n_tiles, tiles * tiles), replace=False))
    tasks, inners, cps = [], [], []
    npix = 0
    for t in pick:
        (y0, y1), (x0, x1) = oracle.tile_bounds(H, tiles)[t // tiles], oracle.tile_bounds(W, tiles)[t % tiles]
        Y0, Y1, X0, X1 = max(y0 - halo, 0), min(y1 + halo, H), max(x0 - halo, 0), min(x1 + halo, W)
        sl = (slice(Y0, Y1), slice(X0, X1))
        inner = ((y0 - Y0, y1 - Y0), (x0 - X0, x1 - X0))
        coords = (xt[X0:X1], yt[Y0:Y1])
        tasks.append(([rr[sl] for rr in fp.ref_raw], fp.sci_raw[sl], fp.dark[sl], fp.flat[sl],
                      fp.bpm[sl], inner, coords, spec_o))
        inners.append(inner)
        cps.append(coords)
        npix += (y1 - y0) * (x1 - x0)
    ctxp = mp.get_context("spawn")
    with ctxp.Pool(cores, initializer=_limit_blas_threads) as pool:
        pool.map(_limit_blas_threads_probe, range(cores))     # workers up before the clock
        t0 = time.perf_counter()
        res = pool.map(_oracle_tile_fit, tasks, chunksize=1)
        A = sum(x[0] for x in res)
        b = sum(x[1] for x in res)
        co, st = oracle.solve(A, b, sum(x[2] for x in res))
        stamps, bg = oracle.expand_kernel(co[None], spec_o)
        res2 = pool.map(_oracle_tile_diff,
                        [(x[3], stamps, bg, inner, cp, spec_o, psf)
                         for x, inner, cp in zip(res, inners, cps)], chunksize=1)
        wall = time.perf_counter() - t0
    pool_rate = npix / wall / 1e6
    # one core, CPU-sized configuration (1024^2 pair, 15x15 constant kernel)
    import threadpoolctl
    c1 = synth.config1_pair(seed=1)
    spec1 = oracle.KernelSpec(half_width=7)
    q = (slice(256, 768), slice(256, 768))          # central 512^2 of the 1024^2 pair
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        cr, vr, mr = oracle.calibrate(c1.ref_raw[0][q], c1.dark[q], c1.flat[q], c1.bpm[q])
        cs, vs, ms = oracle.calibrate(c1.sci_raw[q], c1.dark[q], c1.flat[q], c1.bpm[q])
        co1, _, _ = oracle.fit_kernel(cr, vr, mr, cs, vs, ms, spec1)
        st1, bg1 = oracle.expand_kernel(co1, spec1)
        D, V, dm, _, _ = oracle.subtract(st1, bg1, cr, vr, mr, cs, vs, ms, spec1)
        oracle.detect(D, V, dm, 5.0, psf)
        t1 = time.perf_counter() - t0
    return {"value": round(pool_rate, 4), "unit": "Mpix/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(pick)} of the {tiles * tiles} sub-tiles ({npix / 1e6:.2f} Mpix) of "
                      f"the same full-frame workload, one worker per core (BLAS 1 thread): "
                      f"5-frame calibration + coadd, D=2 h=10 fit (tile normal equations, one "
                      f"FP64 solve), subtraction and detection; {wall:.1f} s wall, status "
                      f"{int(st)}, {sum(res2)} candidates",
            "one_core_config1": {"value": round(512 * 512 / t1 / 1e6, 4), "unit": "Mpix/s",
                                 "s": round(t1, 2),
                                 "workload": "central 512^2 of the 1024^2 CPU-sized pair: calibrate "
                                             "both, 15x15 constant kernel (32 unknowns), subtract, "
                                             "detect; one process, BLAS 1 thread"}}


def _limit_blas_threads_probe(_):
    return os.getpid()


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
    cand_ms, _ = b.tuning()
    shapes = [argus.batch_candidate(i) for i in range(ncand)]
    # the untuned shape: 16-row tiles at the 2 workgroups per CU the kernel's
    # launch bounds are written for
    fixed = shapes.index((16, 2))
    # a second plan of the same problem on this context takes the stored choice
    b2 = argus.Batch(ctx, spec, fr, xs0, ys0, Ls, [W] * nf, [H] * nf)
    ctx.batch_run(b2, frames, 5.0, *outs)
    torch.cuda.synchronize()
    _, hit2 = b2.tuning()
    same2 = b2.info()[0] == choice
    b2.close()
    res = {"value": round(gpix * 1e6 / ms, 2), "unit": "Mpix/s", "ms": round(ms, 3),
           "cutouts": n, "frames": nf, "cutout_gpix": round(gpix, 4),
           "side_px": [int(min(Ls)), int(max(Ls))], "solves_ok": int((st == 0).sum()),
           "autotune": {"choice": choice, "candidates": ncand, "best_ms": round(tuned_ms, 3),
                        "candidate_ms": {f"{t}rows_x{w}wg": round(m, 3)
                                         for (t, w), m in zip(shapes, cand_ms)},
                        "fixed_shape": "16rows_x2wg", "fixed_ms": round(cand_ms[fixed], 3),
                        "gain_vs_fixed": round(cand_ms[fixed] / tuned_ms, 3),
                        "second_plan_from_cache": bool(hit2 and same2)},
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
    # the kernels run only on a tile's valid stamps (the rest of its 64 slots
    # are skipped), so the work is counted on those
    stamps_per_sample = float(V.float().sum(1).mean())
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
    # MACs per valid stamp (961 px, 32 output channels): forward 18 + 3 x 288
    # per pixel and channel, the same again for the weight gradients, and
    # 3 x 288 for the data gradients of layers 3..1
    mac_stamp = 961 * 32 * (2 * (18 + 3 * 288) + 3 * 288)
    train_tflops = samples_s * stamps_per_sample * mac_stamp * 2 / 1e12
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
    # sparse tiles: the same conditions with 300 stars per 1024^2 frame (~19
    # per tile, against ~190): the gain is the kernel error against the fit
    # on the noise-free frames, where that fit exists
    sparse = [sur.Frame(ctx, W, H, 300, 9100 + i, cond, noise_free=True) for i in range(4)]
    rows_sp = sur.evaluate(ctx, path, sparse, B)
    del sparse
    sp_truth = [r for r in rows_sp if r["truth_status"] == 0]
    sp_ok = [r for r in sp_truth if r["plain_status"] == 0]
    sp_failed = [r for r in sp_truth if r["plain_status"] != 0]
    smed = lambda rs, k: (round(float(np.nanmedian([r[k] for r in rs])), 4) if rs else None)
    sparse_res = {"stars_per_frame": 300, "tiles": len(rows_sp),
                  "noise_free_fit_ok": len(sp_truth), "plain_fit_failed": len(sp_failed),
                  "acceptance": (round(float(np.mean([r["accepted"] for r in sp_ok])), 3)
                                 if sp_ok else None),
                  "kernel_err_vs_noise_free": {"plain": smed(sp_ok, "err_plain"),
                                               "surrogate": smed(sp_ok, "err_sur"),
                                               "surrogate_where_plain_failed":
                                                   smed(sp_failed, "err_sur")},
                  "model_err_vs_noise_free": {"plain": smed(sp_ok, "model_err_plain"),
                                              "surrogate": smed(sp_ok, "model_err_sur")},
                  "surrogate_better_frac": (round(float(np.mean([r["err_sur"] < r["err_plain"]
                                                                for r in sp_ok])), 3)
                                            if sp_ok else None)}
    res = {"train": {"samples": n, "frames": args.sur_frames, "epochs": args.sur_epochs,
                     "generate_s": round(t_gen, 2), "samples_per_s": round(samples_s, 1),
                     "valid_stamps_per_sample": round(stamps_per_sample, 2),
                     "stamps_per_s": round(samples_s * stamps_per_sample, 0),
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
           "sparse": sparse_res,
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
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    # per-kernel device times: HIP events around every launch on the launch
    # stream, recorded without synchronisation during the timed steps; one
    # event between consecutive steps gives each step's time
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    step_ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)]
    ms = float(np.median(step_ms))
    ms_mean = ev[0].elapsed_time(ev[-1]) / args.steps
    npix = W * H
    log(f"timed {args.steps} steps: median {ms:.3f} ms/step, mean {ms_mean:.3f} "
        f"(wall {wall:.2f} s)")

    names = ["calibrate", "calibrate_coadd", "fit_accum", "fit_reduce", "fit_solve",
             "subtract", "detect_map", "detect_emit"]
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
            if kind == "alu":
                # against the published FP32 vector peak (which counts packed FP32)
                stages[n]["frac_published_157"] = round(work / t / 1e9 / PEAK_FP32_PUBLISHED, 4)
        else:
            stages[n] = {"ms": round(t, 4)}
    if "detect_map" in kt and "detect_emit" in kt:
        # the whole argus_detect call: map, scan and candidate emission
        t = kt["detect_map"] + kt["detect_emit"]
        work = algorithmic_work("detect_map", spec, npix, 5)[1]
        stages["detect"] = {"ms": round(t, 4), "GB/s": round(work / t / 1e6, 1),
                            "frac_hbm": round(work / t / 1e6 / PEAK_HBM_GBS, 4)}
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
                                   spatial_degree=2, bg_degree=2)
        cpu = cpu_baseline(fp, spec_o, args.cpu_tiles)
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

    # host-to-device copy of one raw frame from pinned memory (reported
    # separately; the step's inputs are resident in HBM)
    host_raw = torch.from_numpy(fp.sci_raw.view(np.int16)).pin_memory()
    dev_raw = torch.empty_like(host_raw, device="cuda")
    h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        dev_raw.copy_(host_raw, non_blocking=True)
    torch.cuda.synchronize()
    h0.record(stream)
    for _ in range(5):
        dev_raw.copy_(host_raw, non_blocking=True)
    h1.record(stream)
    torch.cuda.synchronize()
    h2d_ms = h0.elapsed_time(h1) / 5
    h2d = {"ms": round(h2d_ms, 4), "GB/s": round(npix * 2 / h2d_ms / 1e6, 1),
           "bytes": npix * 2, "workload": "one raw u16 frame, pinned host to device"}
    log("h2d: " + json.dumps(h2d))
    del host_raw, dev_raw

    # background map and source detection on the calibrated science frame
    box = 64
    gx, gy = -(-W // box), -(-H // box)
    grid = torch.empty((gy, gx), dtype=torch.float32, device="cuda")
    bmap = torch.empty((H, W), dtype=torch.float32, device="cuda")
    scap = 262144
    srcs = torch.empty(scap * argus.SOURCE_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    nsrc = torch.empty(1, dtype=torch.int32, device="cuda")
    psf_d = torch.as_tensor(psf.astype(np.float32), device="cuda")

    def sources():
        ctx.background(pipe.sci, pipe.sci_mask, box, grid)
        ctx.detect_sources(pipe.sci, pipe.sci_var, pipe.sci_mask, grid, box, 5.0, psf_d, 7,
                           pipe.snr, pipe.det_mask, srcs, scap, nsrc)

    for _ in range(2):
        sources()
        ctx.background(pipe.sci, pipe.sci_mask, box, grid, bg_map=bmap)
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for _ in range(args.steps):
        sources()
        ctx.background(pipe.sci, pipe.sci_mask, box, grid, bg_map=bmap)
    torch.cuda.synchronize()
    bt = {n: float(ctx.kernel_time_ms(n)) for n in ("background", "background_map", "source_map",
                                                     "source_emit")}
    ctx.set_timing(False)
    bgs = {}
    for n, t, work in (("background", bt["background"], 5.0 * npix),
                       ("background_map", bt["background_map"], 4.0 * npix),
                       ("source_map", bt["source_map"], 14.0 * npix),
                       ("source_detection", bt["source_map"] + bt["source_emit"], 14.0 * npix)):
        bgs[n] = {"ms": round(t, 4), "GB/s": round(work / t / 1e6, 1),
                  "frac_hbm": round(work / t / 1e6 / PEAK_HBM_GBS, 4)}
    bgs["sources"] = int(nsrc.item())
    bgs["workload"] = (f"calibrated science frame: 64x64 cell medians + 3x3 median filter "
                       f"(5 B/px read), full-resolution map (4 B/px written), sources at 5 sigma "
                       f"on cal - background with the calibration variance (14 B/px)")
    log("background/sources: " + json.dumps(bgs))

    # matched-filter coadd of the five reference frames (f3): each calibrated
    # into its own planes, its background grid, one PSF per frame
    t_c = {}
    cal5 = []
    for raw in refs:
        c = torch.empty((H, W), dtype=torch.float32, device="cuda")
        v = torch.empty_like(c)
        m = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        pipe.calibrate(raw, c, v, m)
        g = torch.empty((gy, gx), dtype=torch.float32, device="cuda")
        ctx.background(c, m, box, g)
        cal5.append((c, v, m, g))
    rm = 7
    psf5 = torch.as_tensor(np.stack([synth.psf_image(rm, 2.0) for _ in refs]).astype(np.float32),
                           device="cuda")
    S = torch.empty((H, W), dtype=torch.float32, device="cuda")
    Sv = torch.empty_like(S)
    Sn = torch.empty_like(S)

    def matched():
        ctx.coadd_matched([x[0] for x in cal5], [x[1] for x in cal5], [x[2] for x in cal5], psf5, rm,
                          S, Sv, Sn, grids=[x[3] for x in cal5], box=box)

    matched()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for _ in range(3):
        matched()
    torch.cuda.synchronize()
    t_m = float(ctx.kernel_time_ms("coadd_matched"))
    ctx.set_timing(False)
    flop = 4.0 * (2 * rm + 1) ** 2 * len(refs) * npix
    matched_res = {"ms": round(t_m, 4), "TFLOP/s": round(flop / t_m / 1e9, 2),
                   "frac_valu_78.6": round(flop / t_m / 1e9 / PEAK_FP32_VALU_TFLOPS, 4),
                   "frac_published_157": round(flop / t_m / 1e9 / PEAK_FP32_PUBLISHED, 4),
                   "Mpix/s": round(npix / t_m / 1e3, 1),
                   "workload": f"5 calibrated 9576x6388 frames with background grids, 15x15 PSF each: "
                               f"score, variance and SNR maps"}
    log("matched coadd: " + json.dumps(matched_res))
    del S, Sv, Sn

    # HEALPix segments of the calibrated science frame (f4): NSIDE 256 tiles
    # of 600 x 600 pixels, a gnomonic frame at 1.38 arcsec/px
    s_ = 1.38 / 3600.0
    wcs = argus.make_wcs(120.0, 35.0, (W - 1) / 2.0, (H - 1) / 2.0,
                         [[-s_ * math.cos(0.4), s_ * math.sin(0.4)],
                          [s_ * math.sin(0.4), s_ * math.cos(0.4)]])
    tiles = torch.as_tensor(argus.healpix_tiles(wcs, W, H, 256, 32), device="cuda")
    nt, mseg = int(tiles.shape[0]), 600
    so = torch.empty((nt, mseg, mseg), dtype=torch.float32, device="cuda")
    sov = torch.empty_like(so)
    som = torch.empty((nt, mseg, mseg), dtype=torch.uint8, device="cuda")

    def segments():
        ctx.resample_healpix(pipe.sci, pipe.sci_var, pipe.sci_mask, wcs, 256, mseg, tiles, so, sov, som)

    segments()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for _ in range(3):
        segments()
    torch.cuda.synchronize()
    t_h = float(ctx.kernel_time_ms("healpix_resample"))
    ctx.set_timing(False)
    nseg = nt * mseg * mseg
    healpix_res = {"ms": round(t_h, 4), "tiles": nt, "segment_px": nseg,
                   "Mpix/s_segments": round(nseg / t_h / 1e3, 1),
                   "GB/s": round(18.0 * nseg / t_h / 1e6, 1),
                   "frac_hbm": round(18.0 * nseg / t_h / 1e6 / PEAK_HBM_GBS, 4),
                   "workload": "calibrated science frame (cal, var, mask) into every NSIDE=256 tile "
                               "it touches, 600x600 HEALPix pixels each, bilinear, FP64 geometry; "
                               "18 B per segment pixel (9 gathered, 9 written)"}
    log("healpix: " + json.dumps(healpix_res))
    del so, sov, som

    # ZOGY on overlapping 512 x 512 tiles covering the frame (f2): new =
    # science minus its background, reference = the coadd minus its background
    L, rz = 512, 7
    stride = L - 4 * rz
    xs0 = list(range(0, max(W - L, 0) + 1, stride)) + ([W - L] if (W - L) % stride else [])
    ys0 = list(range(0, max(H - L, 0) + 1, stride)) + ([H - L] if (H - L) % stride else [])
    org = torch.as_tensor(np.array([[x, y] for y in ys0 for x in xs0], np.int32), device="cuda")
    nz = int(org.shape[0])
    gref = torch.empty((gy, gx), dtype=torch.float32, device="cuda")
    ctx.background(pipe.ref, pipe.ref_mask, box, gref)
    ctx.background(pipe.sci, pipe.sci_mask, box, grid)
    bref = torch.empty((H, W), dtype=torch.float32, device="cuda")
    ctx.background(pipe.sci, pipe.sci_mask, box, grid, bg_map=bmap)
    ctx.background(pipe.ref, pipe.ref_mask, box, gref, bg_map=bref)
    Nz = pipe.sci - bmap
    Rz = pipe.ref - bref
    del bref
    Pn = synth.psf_image(rz, 2.6)
    Pr = synth.psf_image(rz, 2.0)
    Pn = torch.as_tensor((Pn / Pn.sum()).astype(np.float32), device="cuda")
    Pr = torch.as_tensor((Pr / Pr.sum()).astype(np.float32), device="cuda")
    sn = float(torch.sqrt(torch.median(pipe.sci_var[pipe.sci_mask == 0])).item())
    sr = float(torch.sqrt(torch.median(pipe.ref_var[pipe.ref_mask == 0])).item())
    zD = torch.empty((nz, L, L), dtype=torch.float32, device="cuda")
    zS, zF = torch.empty_like(zD), torch.empty_like(zD)
    zM = torch.empty((nz, L, L), dtype=torch.uint8, device="cuda")

    def zogy_all():
        ctx.zogy(Nz, pipe.sci_mask, Rz, pipe.ref_mask, org, L, Pn, Pr, rz, 1.05, 1.0, sn, sr,
                 zD, zS, zF, zM)

    zogy_all()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    for _ in range(2):
        zogy_all()
    torch.cuda.synchronize()
    t_z = float(ctx.kernel_time_ms("zogy"))
    ctx.set_timing(False)
    zogy_res = {"ms": round(t_z, 3), "tiles": nz, "tile_px": L, "ms_per_tile": round(t_z / nz, 4),
                "Mpix/s_frame": round(npix / t_z / 1e3, 1),
                "paper_cpu_ms_per_tile": 1400.0,
                "workload": f"{nz} overlapping {L}x{L} tiles (stride {stride}) covering the frame, "
                            f"FP64 transforms, science vs 5-frame coadd, 15x15 PSFs"}
    log("zogy: " + json.dumps(zogy_res))
    del zD, zS, zF, zM, Nz, Rz, cal5


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
    variants = {"precision": prec, "h2d_copy": h2d, "background_and_sources": bgs,
                "matched_coadd": matched_res, "healpix_segments": healpix_res, "zogy": zogy_res,
                "per_frame_difference": {
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
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "ms_per_step_mean": round(ms_mean, 4),
        "higher_is_better": True,
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
