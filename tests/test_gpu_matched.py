"""GPU parity of the matched-filter coadd (argus_coadd_matched) against the
FP64 oracle (oracle/matched.py): five registered exposures with their own
PSFs, variances, masks, flux zero points and background grids (from
argus_background), ragged tiles and a padded pitch.  Bars: score_var relative
<= 1e-5; SNR within 1e-4 absolute plus 1e-6 relative; the flux estimate
score/score_var within 1e-4 of its error plus 1e-5 relative (FP32 outputs)."""
import numpy as np
import pytest

import oracle
from oracle import background as bk
from oracle import matched
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


def _frames(W, H, n, seed):
    fp = synth.make_pair(W, H, 300, seed, 2.0, 2.6, n_ref=n, realistic_masters=True,
                         n_transients=0, cosmic_rate=1e-4)
    out = []
    for j, raw in enumerate(fp.ref_raw):
        c, v, m = oracle.calibrate(raw, fp.dark, fp.flat, fp.bpm)
        out.append((c.astype(np.float32), v.astype(np.float32), m))
    return out


@pytest.mark.parametrize("W,H,r,pad,use_bg", [(700, 500, 7, 0, True), (333, 190, 3, 9, False),
                                              (260, 140, 10, 0, True)])
def test_matched_coadd_matches_oracle(ctx, W, H, r, pad, use_bg):
    import torch
    n = 5
    fr = _frames(W, H, n, 30 + r)
    psfs = np.stack([synth.psf_image(r, 1.8 + 0.3 * j) for j in range(n)]).astype(np.float32)
    scales = [1.0, 0.9, 1.1, 0.95, 1.05]
    box = 32
    d = [[dev(p) for p in f] for f in fr]
    if pad:
        d = [[padded(t, pad) for t in f] for f in d]
    grids, omaps = [], []
    for (c, v, m), (dc, dv, dm) in zip(fr, d):
        if use_bg:
            g = empty((-(-H // box), -(-W // box)), torch.float32)
            ctx.background(dc, dm, box, g)
            grids.append(g)
            omaps.append(bk.background_map(host(g).astype(np.float64), W, H, box))
        else:
            grids.append(None)
            omaps.append(None)
    S = empty((H, W), torch.float32) if not pad else padded(empty((H, W), torch.float32), pad)
    V = empty((H, W), torch.float32) if not pad else padded(empty((H, W), torch.float32), pad)
    N = empty((H, W), torch.float32) if not pad else padded(empty((H, W), torch.float32), pad)
    ctx.coadd_matched([x[0] for x in d], [x[1] for x in d], [x[2] for x in d], dev(psfs), r,
                      S, V, N, grids=grids, box=box, scales=scales)
    oS, oV, oN = matched.matched_coadd([f[0] for f in fr], [f[1] for f in fr], [f[2] for f in fr],
                                       omaps, [p.astype(np.float64) for p in psfs], scales)
    gS, gV, gN = host(S), host(V), host(N)
    pos = oV > 0
    assert np.array_equal(gV > 0, pos)
    vrel = np.abs(gV[pos] / oV[pos] - 1).max()
    serr = np.abs(gN[pos] - oN[pos]) - 1e-6 * np.abs(oN[pos])
    of = oS[pos] / oV[pos]
    ferr = (np.abs(gS[pos] / gV[pos] - of) - 1e-5 * np.abs(of)) * np.sqrt(oV[pos])
    print(f"{W}x{H} r={r}: Var rel {vrel:.2e}, SNR err {serr.max():.2e}, flux err/sigma {ferr.max():.2e}")
    assert vrel <= 1e-5
    assert serr.max() <= 1e-4
    assert ferr.max() <= 1e-4
    assert np.all(gN[~pos] == 0)


def test_matched_rejects_bad_arguments(ctx):
    import torch
    fr = _frames(64, 48, 1, 3)
    d = [dev(p) for p in fr[0]]
    out = empty((48, 64), torch.float32)
    psf = dev(synth.psf_image(11, 2.0).astype(np.float32))
    with pytest.raises(argus.ArgusError):
        ctx.coadd_matched([d[0]], [d[1]], [d[2]], psf, 11, out, out)      # psf_half 11
    with pytest.raises(argus.ArgusError):
        ctx.coadd_matched([d[0]] * 9, [d[1]] * 9, [d[2]] * 9, psf, 3, out, out)
