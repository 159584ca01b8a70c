"""Edge cases of the frame calls on the GPU against the FP64 oracle.

* empty frames (zero rows or columns) are rejected on the host with ESHAPE
  by every frame call, before any launch;
* the largest kernel, h = 15 (31 x 31 stamps), with a linearly varying
  kernel: the fit against the oracle's (stamp bar: the noisy-data bar of the
  h = 7 standard scaled by the ratio of the Jacobi-scaled condition numbers,
  as for the other basis layouts) and the subtraction with the oracle's
  stamps (the stage bars);
* a row pitch larger than the width (13 elements of padding) for the fit,
  the subtraction and the detection: every output is bit-identical to the
  contiguous layout's.
"""
import numpy as np
import pytest

import oracle
from paper_2207_14304_amd import argus, synth
from gpu_util import dev, host, empty, padded
from test_gpu_stages import (NOISY_CHI2_TOL, NOISY_STAMP_TOL, _check_subtract, _det_inputs, _fit,
                             _jacobi_cond, _noisy_pair, _ospec, _run_subtract, _spec)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = argus.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("shape", [(0, 64), (64, 0)])
def test_empty_frames_are_rejected(ctx, shape):
    import torch
    H, W = shape
    f = empty((H, W), torch.float32)
    m = empty((H, W), torch.uint8)
    r = empty((H, W), torch.uint16)
    spec = _spec(half_width=7)
    n, ns = argus.kernel_dims(spec)
    calls = [
        lambda: ctx.calibrate(r, f, f, m, 1.0, 1.7, 65535, f, f, m),
        lambda: ctx.coadd([f] * 3, [f] * 3, [m] * 3, 3.0, 5, f, f, m),
        lambda: ctx.fit_kernel(spec, f, f, m, f, f, m, empty((ns, n), torch.float64),
                               empty(ns, torch.int64), empty(ns, torch.int32)),
        lambda: ctx.subtract(spec, empty((1, 1, 15, 15), torch.float32), empty((1, 1), torch.float32),
                             f, f, m, f, f, m, f, f, m),
        lambda: ctx.detect(f, f, m, 5.0, dev(synth.psf_image(3, 2.6), np.float32), 3, f, m,
                           empty(64 * argus.CANDIDATE_DTYPE.itemsize, torch.uint8), 64,
                           empty(1, torch.int32)),
    ]
    for call in calls:
        with pytest.raises(argus.ArgusError) as e:
            call()
        assert e.value.code == argus.ESHAPE


@pytest.mark.parametrize("prec", [argus.FP32, argus.FP64])
def test_largest_kernel_fit_and_subtraction(ctx, prec):
    h = 15
    planes = _noisy_pair(240, 210, 151, n_stars=220)
    spec = _spec(half_width=h, spatial_degree=1, bg_degree=1, precision=prec)
    os_ = _ospec(spec)
    co, nf, st, stamps, bg, _ = _fit(ctx, spec, planes)
    oco, ost, onf = oracle.fit_kernel(*planes, os_)
    assert st[0] == 0 and ost[0] == 0 and nf[0] == onf[0]
    o_stamps, o_bg = oracle.expand_kernel(oco, os_)
    assert stamps.shape == o_stamps.shape == (1, 3, 2 * h + 1, 2 * h + 1)
    err = np.abs(stamps - o_stamps).max() / np.abs(o_stamps).max()
    std = _ospec(_spec(half_width=7, spatial_degree=1, bg_degree=1))
    ratio = max(1.0, _jacobi_cond(planes, os_) / _jacobi_cond(planes, std))
    gc2 = oracle.chi2(*planes, os_, co)
    oc2 = oracle.chi2(*planes, os_, oco)
    print(f"h=15 prec {prec}: stamp error {err:.3e}, condition ratio {ratio:.1f}, "
          f"chi2 ratio - 1 {gc2[0] / oc2[0] - 1:.3e}")
    assert err <= NOISY_STAMP_TOL[prec] * ratio
    assert abs(gc2[0] / oc2[0] - 1) <= NOISY_CHI2_TOL[prec]
    # the subtraction with the oracle's stamps, against the oracle's
    st32 = o_stamps.astype(np.float32).astype(np.float64)
    bg32 = o_bg.astype(np.float32)
    g = _run_subtract(ctx, spec, st32, bg32, planes)
    o = oracle.subtract(st32, bg32, *planes, os_)
    _check_subtract(g, o)


def test_padded_pitch_is_bit_identical(ctx):
    import torch
    planes = _noisy_pair(203, 177, 77, n_stars=160)
    spec = _spec(half_width=7, spatial_degree=2, bg_degree=2, tiles_x=2, tiles_y=2)
    n, ns = argus.kernel_dims(spec)
    H, W = planes[0].shape
    pad = 13

    def run(pd):
        lay = (lambda t: padded(t, pd)) if pd else (lambda t: t)
        d = [lay(dev(p)) for p in planes]
        co = empty((ns, n), torch.float64)
        nf = empty(ns, torch.int64)
        st = empty(ns, torch.int32)
        ctx.fit_kernel(spec, *d, co, nf, st)
        K = 2 * spec.half_width + 1
        stamps = empty((ns, 6, K, K), torch.float32)
        bg = empty((ns, 6), torch.float32)
        ctx.expand_kernel(spec, co, stamps, bg)
        D = lay(empty((H, W), torch.float32))
        V = lay(empty((H, W), torch.float32))
        M = lay(empty((H, W), torch.uint8))
        c2 = empty(ns, torch.float64)
        nc = empty(ns, torch.int64)
        ctx.subtract(spec, stamps, bg, *d, D, V, M, c2, nc)
        Dd, Vd, Md, P = _det_inputs(W, H, 5)
        snr = lay(empty((H, W), torch.float32))
        det = lay(empty((H, W), torch.uint8))
        cap = 1024
        cands = empty(cap * argus.CANDIDATE_DTYPE.itemsize, torch.uint8)
        ncand = empty(1, torch.int32)
        ctx.detect(lay(dev(Dd)), lay(dev(Vd)), lay(dev(Md)), 5.0, dev(P, np.float32), 5, snr, det,
                   cands, cap, ncand)
        k = int(host(ncand)[0])
        return dict(co=host(co), st=host(st), D=host(D), V=host(V), M=host(M), c2=host(c2),
                    nc=host(nc), snr=host(snr), det=host(det),
                    cands=host(cands)[: k * argus.CANDIDATE_DTYPE.itemsize].copy())

    a, b = run(0), run(pad)
    assert np.all(a["st"] == 0) and a["nc"].sum() > 0 and len(a["cands"]) > 0
    for key in a:
        assert np.array_equal(a[key].view(np.uint8), b[key].view(np.uint8)), key
