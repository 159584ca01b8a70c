"""Batched cutouts in one persistent, graph-captured launch, against the FP64
oracle run on each cutout as a standalone image (fit, expand, subtract,
detect with a constant 15x15 kernel), plus batch-equivalence and
graph-replay determinism.  Bars: with FP64 row moments stamps
max|dK|/max|K| <= 1e-4 and difference RMS <= 1e-4 sigma; with FP32 row
moments (small systems amplify their rounding) 3e-3 and 1e-3 sigma; both:
difference max <= 1e-2 sigma, masks bit-exact, chi^2 relative <= 1e-5.  Cutout sides are drawn log-uniform (ragged sizes,
several tiles each) from three cameras' frames with different seeing."""
import json

import numpy as np
import pytest

import oracle
from paper_2207_14304_amd import argus, synth
from gpu_util import dev, host, empty

pytestmark = pytest.mark.gpu

H_K = 7


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = argus.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def frames():
    out = []
    for i, (W, H, fw) in enumerate([(700, 520, 2.2), (640, 600, 3.1), (560, 500, 1.8)]):
        fp = synth.make_pair(W, H, 500, 40 + i, fw * 2.0 / 2.6, fw, n_transients=5)
        cs, vs, ms = oracle.calibrate(fp.sci_raw, fp.dark, fp.flat, fp.bpm)
        cr, vr, mr = oracle.calibrate(fp.ref_raw[0], fp.dark, fp.flat, fp.bpm)
        rng = np.random.default_rng(i)
        mr[rng.random(mr.shape) < 2e-4] |= oracle.SAT
        ms[rng.random(ms.shape) < 5e-4] |= oracle.BAD
        f = lambda a: a.astype(np.float32)
        out.append(dict(host=(f(cr), f(vr), mr, f(cs), f(vs), ms), fp=fp))
    return out


def _cutouts(frames, n_per, seed, lmin=40, lmax=240):
    fr, x0, y0, L = [], [], [], []
    for i, f in enumerate(frames):
        fp = f["fp"]
        a, b, c = synth.draw_cutouts(seed + i, fp.W, fp.H, fp.star_x, fp.star_y, n_per, lmin, lmax)
        fr += [i] * len(a)
        x0 += list(a)
        y0 += list(b)
        L += list(c)
    return np.array(fr), np.array(x0), np.array(y0), np.array(L)


def _spec(precision=argus.FP64):
    return argus.make_spec(half_width=H_K, precision=precision)


def _run(ctx, frames, cut, reps=1, precision=argus.FP64, between=None):
    import torch
    fr, x0, y0, L = cut
    spec = _spec(precision)
    b = argus.Batch(ctx, spec, fr, x0, y0, L, [f["fp"].W for f in frames],
                    [f["fp"].H for f in frames])
    dframes = [tuple(dev(p) for p in f["host"]) for f in frames]
    n = b.n
    outs = dict(diff=empty(b.arena, torch.float32), var=empty(b.arena, torch.float32),
                mask=empty(b.arena, torch.uint8), det=empty(b.arena, torch.uint8),
                coeffs=empty((n, 32), torch.float64), chi2=empty(n, torch.float64),
                n_fit=empty(n, torch.int64), status=empty(n, torch.int32),
                n_cands=empty(n, torch.int32))
    results = []
    for rep in range(reps):
        if between is not None:
            between(rep)
        ctx.batch_run(b, dframes, 5.0, outs["diff"], outs["var"], outs["mask"], outs["det"],
                      outs["coeffs"], outs["chi2"], outs["n_fit"], outs["status"],
                      outs["n_cands"])
        torch.cuda.synchronize()
        results.append({k: host(v).copy() for k, v in outs.items()})
        # eager work on the caller's stream between replays
        _ = (outs["diff"][:1000] * 2).sum().item()
    return b, results


def _oracle_cutout(frames, fi, x0, y0, L):
    cr, vr, mr, cs, vs, ms = frames[fi]["host"]
    sl = (slice(y0, y0 + L), slice(x0, x0 + L))
    planes = [p[sl] for p in (cr, vr, mr, cs, vs, ms)]
    spec = oracle.KernelSpec(half_width=H_K)
    co, st, nf = oracle.fit_kernel(*planes, spec)
    stamps, bg = oracle.expand_kernel(co, spec)
    D, V, dm, c2, n2 = oracle.subtract(stamps, bg, *planes, spec)
    snr, det, cands = oracle.detect(D, V, dm, 5.0, np.ones((1, 1)))
    return dict(co=co[0], st=st[0], nf=nf[0], stamps=stamps[0, 0], D=D, V=V, dm=dm, c2=c2[0],
                det=det, snr=snr, ncand=len(cands))


# Bars per precision of the row moments.  The small cutouts' systems (down to
# about 700 fit pixels for 32 unknowns) amplify the FP32 rounding of the basis
# convolutions (both precisions) and of the moments (FP32 only): FP64 moments
# keep the difference within 1e-4 sigma RMS (measured <= 2e-5) with stamps
# within 1e-4 (measured <= 6e-5); FP32 moments reach 5e-4 sigma RMS on the
# smallest cutouts, so their bar is 1e-3 sigma RMS, stamps 3e-3.
STAMP_TOL = {argus.FP64: 1e-4, argus.FP32: 3e-3}
RMS_TOL = {argus.FP64: 1e-4, argus.FP32: 1e-3}
VAR_TOL = {argus.FP64: 1e-5, argus.FP32: 3e-4}       # V carries the kernel's error


@pytest.mark.parametrize("precision", [argus.FP64, argus.FP32])
def test_batch_matches_oracle_per_cutout(ctx, frames, precision):
    cut = _cutouts(frames, 8, 100)
    b, (res,) = _run(ctx, frames, cut, precision=precision)
    fr, x0, y0, L = cut
    ospec = oracle.KernelSpec(half_width=H_K)
    B = oracle.basis(ospec)
    rows = []
    for i in range(b.n):
        o = _oracle_cutout(frames, fr[i], x0[i], y0[i], L[i])
        assert res["status"][i] == o["st"] == 0
        assert res["n_fit"][i] == o["nf"]
        off, n2 = b.offsets[i], L[i] * L[i]
        gD = res["diff"][off:off + n2].reshape(L[i], L[i])
        gV = res["var"][off:off + n2].reshape(L[i], L[i])
        gM = res["mask"][off:off + n2].reshape(L[i], L[i])
        gdet = res["det"][off:off + n2].reshape(L[i], L[i])
        gst = np.tensordot(res["coeffs"][i][:31], B, 1)
        ok = o["dm"] == 0
        err = (gD[ok] - o["D"][ok]) / np.sqrt(o["V"][ok])
        near = np.abs(o["snr"] - 5.0) <= 1e-3
        rows.append(dict(L=int(L[i]), nf=int(o["nf"]),
                         stamp=float(np.abs(gst - o["stamps"]).max() / np.abs(o["stamps"]).max()),
                         rms=float(np.sqrt(np.mean(err ** 2))), mx=float(np.abs(err).max()),
                         var=float(np.abs(gV[ok] / o["V"][ok] - 1).max()),
                         chi2=float(abs(res["chi2"][i] / o["c2"] - 1)),
                         mask=bool(np.array_equal(gM, o["dm"])),
                         det=bool(np.array_equal(gdet[~near], o["det"][~near])),
                         cand=bool(near.any() or res["n_cands"][i] == o["ncand"])))
    for r in rows:
        print(r)
    for r in rows:
        assert r["mask"] and r["det"] and r["cand"], r
        assert r["stamp"] <= STAMP_TOL[precision], r
        assert r["rms"] <= RMS_TOL[precision] and r["mx"] <= 1e-2, r
        assert r["var"] <= VAR_TOL[precision] and r["chi2"] <= 1e-5, r


def test_batch_equivalence_and_graph_replays(ctx, frames):
    """A cutout processed in a batch and alone gives bit-identical outputs, and
    every graph replay reproduces the first (autotuning) run bit for bit."""
    cut = _cutouts(frames, 12, 200)
    b, res = _run(ctx, frames, cut, reps=3)
    for r in res[1:]:
        for k in res[0]:
            assert np.array_equal(r[k], res[0][k]), k
    choice, ms, ncand = b.info()
    assert 0 <= choice < ncand and ms > 0
    fr, x0, y0, L = cut
    for i in (0, 5, len(L) - 1):
        b1, (r1,) = _run(ctx, frames, (fr[i:i + 1], x0[i:i + 1], y0[i:i + 1], L[i:i + 1]))
        off, n2 = b.offsets[i], L[i] * L[i]
        assert np.array_equal(r1["coeffs"][0], res[0]["coeffs"][i])
        for k in ("diff", "var", "mask", "det"):
            assert np.array_equal(r1[k][:n2], res[0][k][off:off + n2]), k
        # the chi^2 sum order follows the autotuned tile height
        assert abs(r1["chi2"][0] / res[0]["chi2"][i] - 1) <= 1e-12


def test_batch_rejects_bad_cutouts(ctx, frames):
    fp = frames[0]["fp"]
    with pytest.raises(argus.ArgusError):
        argus.Batch(ctx, _spec(), [0], [fp.W - 10], [0], [64], [fp.W], [fp.H])
    with pytest.raises(argus.ArgusError):
        argus.Batch(ctx, _spec(), [1], [0], [0], [64], [fp.W], [fp.H])
    with pytest.raises(argus.ArgusError):
        argus.Batch(ctx, argus.make_spec(half_width=7, spatial_degree=1), [0], [0], [0], [64],
                    [fp.W], [fp.H])


def test_batch_keeps_its_basis_across_other_fits(ctx, frames):
    """The captured graph reads the basis tables of the batch's own plan.
    Fits and kernel expansions with other specs on the same context (21x21
    degree-2 and 11x11 constant kernels rebuild the context's tables) between
    the plan and the first run and between graph replays change none of the
    batch's outputs, which still match the oracle."""
    import torch
    cut = _cutouts(frames, 6, 300)
    _, (clean,) = _run(ctx, frames, cut)
    dplanes = [dev(p) for p in frames[0]["host"]]
    specs = [argus.make_spec(half_width=10, spatial_degree=2, bg_degree=2),
             argus.make_spec(half_width=5)]

    def other_fit(rep):
        spec = specs[rep % 2]
        n, ns = argus.kernel_dims(spec)
        co = empty((ns, n), torch.float64)
        ctx.fit_kernel(spec, *dplanes, co, empty(ns, torch.int64), empty(ns, torch.int32))
        nP = 6 if rep % 2 == 0 else 1
        K = 2 * spec.half_width + 1
        ctx.expand_kernel(spec, co, empty((ns, nP, K, K), torch.float32),
                          empty((ns, nP), torch.float32))

    b, res = _run(ctx, frames, cut, reps=3, between=other_fit)
    for r in res:
        for k in clean:
            if k == "chi2":       # its sum order follows the autotuned tile height
                assert np.allclose(r[k], clean[k], rtol=1e-12, atol=0), k
            else:
                assert np.array_equal(r[k], clean[k]), k
    fr, x0, y0, L = cut
    ospec = oracle.KernelSpec(half_width=H_K)
    B = oracle.basis(ospec)
    for i in (0, b.n - 1):
        o = _oracle_cutout(frames, fr[i], x0[i], y0[i], L[i])
        gst = np.tensordot(res[-1]["coeffs"][i][:31], B, 1)
        assert np.abs(gst - o["stamps"]).max() <= STAMP_TOL[argus.FP64] * np.abs(o["stamps"]).max()
        off, n2 = b.offsets[i], L[i] * L[i]
        gD = res[-1]["diff"][off:off + n2].reshape(L[i], L[i])
        ok = o["dm"] == 0
        err = (gD[ok] - o["D"][ok]) / np.sqrt(o["V"][ok])
        assert np.sqrt(np.mean(err ** 2)) <= RMS_TOL[argus.FP64]


def test_batch_tuning_cache(frames, tmp_path):
    """The autotuner's outcome (choice and every candidate's time) is stored
    under a key naming the device, the HIP runtime, the kernel and the size
    bucket, in a JSON-lines file; a new context reading that file takes the
    stored choice without timing and gives bit-identical outputs."""
    path = tmp_path / "tune.jsonl"
    path.write_text("not an entry\n")             # lines that do not parse are skipped
    cut = _cutouts(frames, 6, 400)
    c1 = argus.Context(0)
    c1.set_tune_cache(path)
    b1, (r1,) = _run(c1, frames, cut)
    ms1, hit1 = b1.tuning()
    choice, best, ncand = b1.info()
    assert not hit1 and len(ms1) == ncand and min(ms1) > 0 and best == ms1[choice] == min(ms1)
    lines = path.read_text().splitlines()
    assert len(lines) == 2
    entry = json.loads(lines[1])
    assert entry["choice"] == choice and len(entry["ms"]) == ncand
    for part in ("device=gfx", ";hip=", ";kernel=batch;h=7;", ";log2n="):
        assert part in entry["key"], entry["key"]
    c2 = argus.Context(0)
    c2.set_tune_cache(path)
    b2, (r2,) = _run(c2, frames, cut)
    ms2, hit2 = b2.tuning()
    assert hit2 and b2.info()[0] == choice and ms2 == pytest.approx(ms1, rel=1e-5)
    for k in r1:
        assert np.array_equal(r1[k], r2[k]), k
    assert len(path.read_text().splitlines()) == 2   # nothing new stored
    for c in (c1, c2):
        c.close()
