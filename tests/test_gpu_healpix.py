"""GPU parity of the HEALPix segment resampling (argus_healpix_tiles,
argus_resample_healpix) against the FP64 oracle (oracle/healpix.py): the
tile list of a rotated gnomonic frame, and every segment pixel's value,
variance and mask.  Bars: tile lists equal; masks bit-exact except where the
oracle's frame position lies within 1e-9 px of a pixel boundary or the frame
edge (counted, expected none); values and variances within 2 FP32 ulp of the
oracle's (FP64 geometry and weights on both sides)."""
import math

import numpy as np
import pytest

import oracle
from oracle import healpix as hp
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


def _wcs_pair(W, H, ra0, dec0, rot, scale=1.38):
    s = scale / 3600.0
    c, t = math.cos(rot), math.sin(rot)
    cd = [[-s * c, s * t], [s * t, s * c]]
    crpix = ((W - 1) / 2.0, (H - 1) / 2.0)
    return hp.Wcs(ra0, dec0, crpix[0], crpix[1], cd), argus.make_wcs(ra0, dec0, crpix[0], crpix[1], cd)


def _ulps(g, o):
    o32 = np.asarray(o, np.float64).astype(np.float32)
    sp = np.spacing(np.abs(o32)).astype(np.float64)
    sp[sp == 0] = np.spacing(np.float32(0))
    return np.abs(np.asarray(g, np.float64) - np.asarray(o, np.float64)) / sp


def _near_boundary(wo, tiles, nside, m, W, H):
    out = []
    for t in tiles:
        x, y, den = hp.segment_positions(wo, tuple(t), nside, m)
        fx, fy = x - np.round(x), y - np.round(y)
        out.append((np.abs(fx) < 1e-9) | (np.abs(fy) < 1e-9) | (np.abs(x) < 1e-9) |
                   (np.abs(x - (W - 1)) < 1e-9) | (np.abs(y) < 1e-9) | (np.abs(y - (H - 1)) < 1e-9))
    return np.array(out)


@pytest.mark.parametrize("W,H,ra0,dec0,rot,pad", [(900, 700, 83.6, 22.0, 0.3, 0),
                                                  (640, 480, 200.0, 75.0, -1.1, 7),
                                                  (700, 500, 45.0, -0.01, 2.0, 0)])
def test_resample_matches_oracle(ctx, W, H, ra0, dec0, rot, pad):
    import torch
    wo, wg = _wcs_pair(W, H, ra0, dec0, rot)
    nside, m = 256, 600
    tiles = argus.healpix_tiles(wg, W, H, nside, 32)
    otiles = hp.tiles_of_frame(wo, W, H, nside)
    assert [tuple(t) for t in tiles.tolist()] == otiles and len(otiles) >= 2
    fp = synth.make_pair(W, H, 300, 5 + W, 2.0, 2.6, n_transients=0, realistic_masters=True)
    cal, var, mask = oracle.calibrate(fp.sci_raw, fp.dark, fp.flat, fp.bpm)
    cal, var = cal.astype(np.float32), var.astype(np.float32)
    dc, dv, dm = dev(cal), dev(var), dev(mask)
    if pad:
        dc, dv, dm = padded(dc, pad), padded(dv, pad), padded(dm, pad)
    n = len(tiles)
    out = empty((n, m, m), torch.float32)
    ov = empty((n, m, m), torch.float32)
    om = empty((n, m, m), torch.uint8)
    ctx.resample_healpix(dc, dv, dm, wg, nside, m, dev(tiles.astype(np.int32)), out, ov, om)
    val, vv, mm = hp.resample(cal, var, mask, wo, otiles, nside, m)
    g, gv, gm = host(out), host(ov), host(om)
    near = _near_boundary(wo, otiles, nside, m, W, H)
    print(f"{W}x{H} at ({ra0}, {dec0}): {n} tiles, {int((mm == 0).sum())} segment pixels with "
          f"data, near-boundary {int(near.sum())}")
    assert near.sum() <= 4
    assert np.array_equal(gm[~near], mm[~near])
    ok = (mm == 0) & (gm == 0)
    assert _ulps(g[ok], val[ok]).max() <= 2 and _ulps(gv[ok], vv[ok]).max() <= 2
    assert np.all(g[gm != 0] == 0) and np.all(gv[gm != 0] == 0)


def test_resample_rejects_bad_arguments(ctx):
    import torch
    wo, wg = _wcs_pair(64, 48, 10.0, 10.0, 0.0)
    t = dev(np.array([[4, 1, 1]], np.int32))
    a = empty((48, 64), torch.float32)
    msk = empty((48, 64), torch.uint8)
    o = empty((1, 8, 8), torch.float32)
    om = empty((1, 8, 8), torch.uint8)
    with pytest.raises(argus.ArgusError):
        ctx.resample_healpix(a, a, msk, wg, 256, 0, t, o, o, om)        # m = 0
    bad = argus.make_wcs(10.0, 10.0, 0.0, 0.0, [[1.0, 2.0], [2.0, 4.0]])   # singular cd
    with pytest.raises(argus.ArgusError):
        ctx.resample_healpix(a, a, msk, bad, 256, 8, t, o, o, om)


def test_full_frame_segments_sampled(ctx):
    """The 9576 x 6388 frame at 1.38 arcsec/px: every tile it touches on the
    GPU, six of them (the first, the last and four at random) against the
    oracle pixel by pixel."""
    import torch
    W, H = 9576, 6388
    wo, wg = _wcs_pair(W, H, 120.0, 35.0, 0.4)
    tiles = argus.healpix_tiles(wg, W, H, 256, 32)
    assert [tuple(t) for t in tiles.tolist()] == hp.tiles_of_frame(wo, W, H, 256)
    rng = np.random.default_rng(8)
    y, x = np.mgrid[0:H, 0:W]
    cal = (800.0 + 30.0 * np.sin(x / 300.0) + rng.standard_normal((H, W)) * 20).astype(np.float32)
    var = np.full((H, W), 400.0, np.float32)
    mask = np.zeros((H, W), np.uint8)
    mask[rng.random((H, W)) < 1e-4] = oracle.BAD
    del x, y
    n, m = len(tiles), 600
    out = empty((n, m, m), torch.float32)
    ov = empty((n, m, m), torch.float32)
    om = empty((n, m, m), torch.uint8)
    ctx.resample_healpix(dev(cal), dev(var), dev(mask), wg, 256, m, dev(tiles), out, ov, om)
    g, gv, gm = host(out), host(ov), host(om)
    covered = int((gm == 0).sum())
    print(f"full frame: {n} tiles, {covered} segment pixels with data ({covered / (W * H):.3f} of "
          f"the frame's pixel count)")
    assert 0.9 < covered / (W * H) < 1.1
    pick = sorted(set([0, n - 1] + list(rng.choice(n, 4, replace=False))))
    for i in pick:
        t = tuple(tiles[i].tolist())
        val, vv, mm = hp.resample(cal, var, mask, wo, [t], 256, m)
        near = _near_boundary(wo, [t], 256, m, W, H)[0]
        assert np.array_equal(gm[i][~near], mm[0][~near])
        ok = (mm[0] == 0) & (gm[i] == 0)
        assert _ulps(g[i][ok], val[0][ok]).max() <= 2 and _ulps(gv[i][ok], vv[0][ok]).max() <= 2
