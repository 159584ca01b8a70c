"""GPU parity of the median-filtered background map and the full-frame
source detection against the FP64 oracle (oracle/background.py).

Bars: cell levels bit-exact against the oracle's medians rounded to FP32 (the
median selects input values; an even count's mean is rounded once), with
the empty cells equal; the filtered grid bit-exact against the oracle's 3 x 3
median of the GPU's levels (and within one FP32 ulp of the oracle's own
chain); the map within 1e-6 of the grid's scale (FP32 interpolation weights);
sources: SNR within 1e-4 absolute plus 1e-6 relative (FP32 rounding of
D/sqrt(V) at the SNR of bright stars), given the same grid; DET/CAND bit-exact except
where the oracle's SNR is within 1e-3 of the threshold or of a neighbour's,
fluxes relative <= 1e-4, centroids within 1e-4 px plus the FP32 spacing of
the stored coordinate (2.4e-4 px at y = 3000).  Frames have ragged last
cells, masked pixels, a fully masked cell and a padded row pitch."""
import numpy as np
import pytest

import oracle
from oracle import background as bk
from paper_2207_14304_amd import argus, synth
from gpu_util import dev, host, empty, padded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = argus.Context(0)
    yield c
    c.close()


def _frame(W, H, seed, n_stars=400):
    fp = synth.make_pair(W, H, n_stars, seed, 2.0, 2.6, n_transients=0, realistic_masters=True)
    cal, var, mask = oracle.calibrate(fp.sci_raw, fp.dark, fp.flat, fp.bpm)
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:H, 0:W]
    cal = cal + 30.0 * np.sin(x / 211.0) + 0.02 * y          # a background worth mapping
    mask[rng.random((H, W)) < 1e-3] |= oracle.SAT
    mask[64:128, 64:128] |= oracle.BAD                        # one whole 64 cell (four 32 cells)
    cal[mask != 0] = 0.0
    return cal.astype(np.float32), var.astype(np.float32), mask


def _near_ties(snr, thr, tol):
    H, W = snr.shape
    near = np.abs(snr - thr) <= tol
    pad = np.full((H + 2, W + 2), -np.inf)
    pad[1:-1, 1:-1] = snr
    close = np.zeros_like(near)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx or dy:
                close |= np.abs(snr - pad[1 + dy:H + 1 + dy, 1 + dx:W + 1 + dx]) <= tol
    return near | (close & (snr >= thr - tol))


def _run(ctx, cal, var, mask, box, pad=0):
    import torch
    H, W = cal.shape
    gx, gy = -(-W // box), -(-H // box)
    dc, dv, dm = dev(cal), dev(var), dev(mask)
    if pad:
        dc, dv, dm = padded(dc, pad), padded(dv, pad), padded(dm, pad)
    lev = empty((gy, gx), torch.float32)
    grid = empty((gy, gx), torch.float32)
    bmap = empty((H, W), torch.float32) if not pad else padded(empty((H, W), torch.float32), pad)
    ctx.background(dc, dm, box, grid, levels=lev, bg_map=bmap)
    P = synth.psf_image(5, 2.6)
    cap = 8192
    snr = empty((H, W), torch.float32) if not pad else padded(empty((H, W), torch.float32), pad)
    det = empty((H, W), torch.uint8) if not pad else padded(empty((H, W), torch.uint8), pad)
    src = empty(cap * argus.SOURCE_DTYPE.itemsize, torch.uint8)
    ns = empty(1, torch.int32)
    ctx.detect_sources(dc, dv, dm, grid, box, 5.0, dev(P, np.float32), 5, snr, det, src, cap, ns)
    n = int(host(ns)[0])
    s = host(src)[: min(n, cap) * argus.SOURCE_DTYPE.itemsize].view(argus.SOURCE_DTYPE)
    return dict(levels=host(lev), grid=host(grid), map=host(bmap), snr=host(snr), det=host(det),
                src=s.copy(), n=n, P=P)


@pytest.mark.parametrize("W,H,box,pad", [(1100, 700, 64, 0), (333, 257, 32, 0),
                                         (520, 390, 64, 13)])
def test_background_and_sources(ctx, W, H, box, pad):
    cal, var, mask = _frame(W, H, 7 + W)
    g = _run(ctx, cal, var, mask, box, pad)
    lev = bk.cell_levels(cal, mask, box)
    # levels: the oracle's medians rounded to FP32, empty cells NaN on both
    assert np.array_equal(np.isnan(g["levels"]), np.isnan(lev)) and np.isnan(lev).any()
    ok = ~np.isnan(lev)
    assert np.array_equal(g["levels"][ok], lev[ok].astype(np.float32))
    # filter: exact on the GPU's levels, within one ulp of the oracle chain
    gl = g["levels"].astype(np.float64)
    assert np.array_equal(g["grid"], bk.median_filter3(gl).astype(np.float32))
    og = bk.median_filter3(lev)
    assert np.all(np.abs(g["grid"] - og) <= np.spacing(np.abs(og).astype(np.float32)))
    # map: the interpolation of the GPU's grid
    om = bk.background_map(g["grid"].astype(np.float64), W, H, box)
    assert np.abs(g["map"] - om).max() <= 1e-6 * np.abs(og).max()
    # sources on D = cal - map
    snr, det, src = bk.detect_sources(cal, var, mask, om, 5.0, g["P"])
    good = mask == 0
    assert np.all(np.abs(g["snr"][good] - snr[good]) <= 1e-4 + 1e-6 * np.abs(snr[good]))
    near = _near_ties(snr, 5.0, 1e-3)
    assert np.array_equal(g["det"][~near], det[~near])
    print(f"{W}x{H} box {box}: {g['n']} sources (oracle {len(src)}), near-ties {int(near.sum())}")
    assert g["n"] == len(src) and g["n"] > 20
    gs = g["src"]
    assert np.array_equal(gs["x"], src["x"]) and np.array_equal(gs["y"], src["y"])
    assert np.allclose(gs["flux"], src["flux"], rtol=1e-4)
    assert np.allclose(gs["flux_err"], src["flux_err"], rtol=1e-4)
    assert np.allclose(gs["snr"], src["snr"], rtol=1e-6, atol=1e-4)
    # centroids: 1e-4 px plus the FP32 spacing of the stored coordinate
    for k in ("xc", "yc"):
        tol = 1e-4 + np.spacing(np.abs(src[k]).astype(np.float32))
        assert np.array_equal(np.isnan(gs[k]), np.isnan(src[k]))
        ok = ~np.isnan(src[k])
        assert np.all(np.abs(gs[k][ok] - src[k][ok]) <= tol[ok]), k


def test_background_rejects_bad_box(ctx):
    import torch
    cal, var, mask = _frame(128, 96, 3, 50)
    grid = empty((48, 64), torch.float32)
    for box in (3, 65):
        with pytest.raises(argus.ArgusError):
            ctx.background(dev(cal), dev(mask), box, grid)


def test_full_frame_background_and_sources(ctx):
    """The whole 9576 x 6388 frame: every cell level and the filtered grid
    against the oracle; sources on the whole frame (positions and SNR), their
    fluxes and centroids at 300 sampled sources."""
    import torch
    W, H, box = 9576, 6388, 64
    rng = np.random.default_rng(17)
    n = 4000
    xs, ys = rng.uniform(0, W, n), rng.uniform(0, H, n)
    fl = synth.draw_fluxes(rng, n, 1e3, 1e6)
    scene = synth.render_scene(W, H, xs, ys, fl, lambda x: np.full(np.shape(x), 2.6))
    y, x = np.mgrid[0:H, 0:W]
    sky = 800.0 + 40.0 * np.sin(x / 900.0) * np.cos(y / 700.0)
    var = (sky + scene + 2.89).astype(np.float32)
    cal = (sky + scene + rng.standard_normal((H, W)) * np.sqrt(var)).astype(np.float32)
    del scene, sky, x, y
    mask = np.zeros((H, W), np.uint8)
    mask[rng.random((H, W)) < 1e-4] = oracle.BAD
    cal[mask != 0] = 0.0
    gx, gy = -(-W // box), -(-H // box)
    dc, dv, dm = dev(cal), dev(var), dev(mask)
    lev = empty((gy, gx), torch.float32)
    grid = empty((gy, gx), torch.float32)
    ctx.background(dc, dm, box, grid, levels=lev)
    olev = bk.cell_levels(cal, mask, box)
    assert np.array_equal(host(lev), olev.astype(np.float32))
    ggrid = host(grid)
    assert np.array_equal(ggrid, bk.median_filter3(olev.astype(np.float32).astype(np.float64))
                          .astype(np.float32))
    P = synth.psf_image(7, 2.6)
    cap = 65536
    snr = empty((H, W), torch.float32)
    det = empty((H, W), torch.uint8)
    src = empty(cap * argus.SOURCE_DTYPE.itemsize, torch.uint8)
    ns = empty(1, torch.int32)
    ctx.detect_sources(dc, dv, dm, grid, box, 5.0, dev(P, np.float32), 7, snr, det, src, cap, ns)
    nsrc = int(host(ns)[0])
    gs = host(src)[: nsrc * argus.SOURCE_DTYPE.itemsize].view(argus.SOURCE_DTYPE)
    om = bk.background_map(ggrid.astype(np.float64), W, H, box)
    D = cal - om
    osnr, odet, oc = oracle.detect(D, var, mask, 5.0, np.ones((1, 1)))   # positions only
    gsnr = host(snr)
    assert np.all(np.abs(gsnr - osnr) <= 1e-4 + 1e-6 * np.abs(osnr))
    near = _near_ties(osnr, 5.0, 1e-3)
    assert np.array_equal(host(det)[~near], odet[~near])
    print(f"full frame: {nsrc} sources, near-ties {int(near.sum())}")
    assert nsrc == len(oc) and nsrc > 2000
    assert np.array_equal(gs["x"], oc["x"]) and np.array_equal(gs["y"], oc["y"])
    for i in rng.choice(nsrc, 300, replace=False):            # flux and centroid by definition
        cx, cy = int(gs["x"][i]), int(gs["y"][i])
        y0, y1, x0, x1 = max(cy - 7, 0), min(cy + 8, H), max(cx - 7, 0), min(cx + 8, W)
        p = P[y0 - cy + 7:y1 - cy + 7, x0 - cx + 7:x1 - cx + 7]
        ok = mask[y0:y1, x0:x1] == 0
        v = var[y0:y1, x0:x1].astype(np.float64)
        q = (p * p / v)[ok].sum()
        f = (p * D[y0:y1, x0:x1] / v)[ok].sum() / q
        assert abs(gs["flux"][i] - f) <= 1e-4 * abs(f) + 1e-3, (i, gs[i], f)
        w = np.maximum(D[max(cy - 1, 0):cy + 2, max(cx - 1, 0):cx + 2], 0.0)
        w = w * (mask[max(cy - 1, 0):cy + 2, max(cx - 1, 0):cx + 2] == 0)
        uu = np.arange(max(cx - 1, 0), min(cx + 2, W)) - cx
        vv = np.arange(max(cy - 1, 0), min(cy + 2, H)) - cy
        xc, yc = cx + (w * uu[None, :]).sum() / w.sum(), cy + (w * vv[:, None]).sum() / w.sum()
        assert abs(gs["xc"][i] - xc) <= 1e-4 + np.spacing(np.float32(xc)), (i, gs[i], xc)
        assert abs(gs["yc"][i] - yc) <= 1e-4 + np.spacing(np.float32(yc)), (i, gs[i], yc)
