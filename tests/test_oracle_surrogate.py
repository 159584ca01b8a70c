"""Pins of the surrogate oracle: convolution against scipy, gradients
against central finite differences, Adam's first step in closed form, stamp
selection and normalisation by brute force, and the background formula on
in-span data."""
import numpy as np
import pytest
from scipy import signal

import oracle
from oracle import surrogate as sg


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((2, 3, 9, 8))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = sg.conv3x3(a, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate2d(a[n, c], w[o, c], mode="same") for c in range(3))
            assert np.allclose(out[n, o], ref, rtol=1e-12, atol=1e-12)


def _tiny():
    rng = np.random.default_rng(1)
    p = sg.init_params(rng, C=4, cin=2, nout=5)
    X = rng.standard_normal((2, 3, 2, 7, 7))
    valid = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 1.0]])
    tgt = rng.standard_normal((2, 5))
    return p, X, valid, tgt


def test_backward_matches_finite_differences():
    p, X, valid, tgt = _tiny()
    out, cache = sg.forward(p, X, valid)
    g = sg.backward(p, cache, out, tgt)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        num = np.zeros_like(flat)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + eps
            lp = sg.loss(sg.forward(p, X, valid)[0], tgt)
            flat[i] = old - eps
            lm = sg.loss(sg.forward(p, X, valid)[0], tgt)
            flat[i] = old
            num[i] = (lp - lm) / (2 * eps)
        ana = g[k].reshape(-1)
        scale = max(np.abs(num).max(), 1e-12)
        assert np.abs(ana - num).max() <= 1e-7 * max(scale, 1.0), k


def test_invalid_stamps_do_not_contribute():
    p, X, valid, tgt = _tiny()
    out, _ = sg.forward(p, X, valid)
    X2 = X.copy()
    X2[0, 2] = 123.0                       # stamp 2 of tile 0 is invalid
    out2, _ = sg.forward(p, X2, valid)
    assert np.array_equal(out, out2)


def _features(p, stamp):
    """Spatial mean of the last layer for one stamp pair, written out with
    scipy's correlation (independent of sg.conv3x3)."""
    a = stamp
    for l in range(4):
        w, b = p[f"w{l}"], p[f"b{l}"]
        a = np.maximum(np.stack([b[o] + sum(signal.correlate2d(a[c], w[o, c], mode="same")
                                            for c in range(a.shape[0]))
                                 for o in range(w.shape[0])]), 0.0)
    return a.mean(axis=(1, 2))


def test_forward_is_the_mean_over_valid_stamps():
    """Closed forms of the pooling over stamps: a tile with one valid stamp
    gives hw . f(s) + hb; k copies of that stamp give the same output
    (the mean divides by the number of valid stamps, not by S); two valid
    stamps give the mean of their features; invalid slots hold garbage."""
    rng = np.random.default_rng(21)
    p = sg.init_params(rng, C=4, cin=2, nout=5)
    for l in range(4):
        p[f"b{l}"] = 0.1 * rng.standard_normal(4)
    p["hb"] = rng.standard_normal(5)
    s0, s1 = rng.standard_normal((2, 2, 7, 7))
    X = 50.0 * rng.standard_normal((3, 4, 2, 7, 7))
    X[0, 2] = s0
    X[1, 0] = X[1, 1] = X[1, 3] = s0
    X[2, 1], X[2, 3] = s0, s1
    valid = np.array([[0, 0, 1, 0], [1, 1, 0, 1], [0, 1, 0, 1]], np.float64)
    out, _ = sg.forward(p, X, valid)
    f0, f1 = _features(p, s0), _features(p, s1)
    assert np.allclose(out[0], p["hw"] @ f0 + p["hb"], rtol=1e-12, atol=1e-12)
    assert np.allclose(out[1], out[0], rtol=1e-12, atol=1e-12)
    assert np.allclose(out[2], p["hw"] @ ((f0 + f1) / 2) + p["hb"], rtol=1e-12, atol=1e-12)


def test_adam_first_step_closed_form():
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -0.25, 0.0])}
    st = {}
    sg.adam_step(p, g, st, lr=0.1)
    exp = np.array([1.0 - 0.1 * 0.5 / (0.5 + 1e-8), -2.0 + 0.1 * 0.25 / (0.25 + 1e-8), 3.0])
    assert np.allclose(p["w"], exp, rtol=1e-12)
    assert st["t"] == 1


def test_stamp_selection_and_normalisation():
    H, W = 60, 70
    ref = np.full((H, W), 10.0)
    var = np.full((H, W), 1.0)
    peaks = [(20, 20, 500.0), (30, 40, 900.0), (3, 30, 2000.0), (40, 22, 900.0), (45, 50, 300.0)]
    for y, x, v in peaks:
        ref[y, x] = v
    rm = np.zeros((H, W), np.uint8)
    sm = np.zeros((H, W), np.uint8)
    sm[45 + 3, 50 - 2] = 1                       # masks the stamp around (45, 50)
    cs = sg.select_stamps(ref, var, rm, sm, 1, 1, r=4, S=3)
    # (3,30) is too close to the edge; (45,50) is masked; equal peaks: raster first
    assert cs == [[(30, 40), (40, 22), (20, 20)]]
    sci = 2.0 * ref + 7.0
    Xs, v = sg.make_stamps(ref, sci, cs, r=4, S=3)
    assert v.tolist() == [[1.0, 1.0, 1.0]]
    assert np.allclose(Xs[0, :, 0].sum(axis=(1, 2)), sg.STAMP_SCALE)
    assert np.allclose(Xs[0, :, 1], 2.0 * Xs[0, :, 0])
    st = np.arange(25.0).reshape(5, 5)
    b = np.r_[st[0], st[-1], st[1:-1, 0], st[1:-1, -1]]
    assert sg.border_median(st) == np.median(b)


def test_background_given_kernel_in_span():
    from test_oracle_pins import _star_ref
    H, W = 60, 64
    ref = _star_ref(W, H, 15, 9)
    spec = oracle.KernelSpec(half_width=4)
    B = oracle.basis(spec)
    K = 1.03 * B[0] + 0.02 * B[3]
    sci = signal.convolve2d(ref, K, mode="same") - 17.5
    one = np.ones((H, W))
    z = np.zeros((H, W), np.uint8)
    bg = sg.background_given_kernel(K, ref, one, z, sci, one, z, 4)
    assert bg == pytest.approx(-17.5, abs=1e-9)


def test_select_per_tile_pins():
    """In span with a per-tile kernel and background the true kernel gets its
    background back with chi^2 = 0; given the plain fit's own kernel the
    one-parameter background equals the joint fit's (its partial derivative
    vanishes at the joint optimum) with the same chi^2, so the tile is kept;
    a kernel scaled by 1.5 is rejected."""
    from test_oracle_pins import _star_ref
    H, W = 64, 72
    ref = _star_ref(W, H, 30, 11)
    spec = oracle.KernelSpec(half_width=4, tiles_x=2, tiles_y=1, mode=oracle.core.PER_TILE)
    B = oracle.basis(spec)
    nb = len(B)
    rng = np.random.default_rng(5)
    one = np.ones((H, W))
    z = np.zeros((H, W), np.uint8)
    true = np.zeros((2, nb))
    true[:, 0] = [1.02, 0.97]
    true[:, 4] = [0.03, -0.02]
    bgs = [12.0, -4.5]
    sci = np.zeros((H, W))
    for t, (x0, x1, y0, y1) in enumerate(oracle.core._solve_regions(spec, W, H)):
        full = signal.convolve2d(ref, np.tensordot(true[t], B, 1), mode="same") + bgs[t]
        sci[y0:y1, x0:x1] = full[y0:y1, x0:x1]
    out, rs, acc = sg.select_per_tile(true, np.zeros((2, nb + 1)), np.ones(2), np.full(2, 10**6),
                                      ref, one, z, sci, one, z, spec)
    assert np.allclose(out[:, nb], bgs, atol=1e-8)
    assert np.all(rs < 1e-14) and acc.all()
    noisy = sci + rng.standard_normal((H, W))
    co, st, nf = oracle.fit_kernel(ref, one, z, noisy, one, z, spec)
    stamps, bgp = oracle.expand_kernel(co, spec)
    _, _, _, c2, n2 = oracle.subtract(stamps, bgp, ref, one, z, noisy, one, z, spec)
    out, rs, acc = sg.select_per_tile(co[:, :nb], co, c2, n2, ref, one, z, noisy, one, z, spec)
    assert np.allclose(out[:, nb], co[:, nb], rtol=1e-9, atol=1e-9)
    assert np.allclose(rs * (n2 - 1), c2, rtol=1e-9)
    assert acc.all()
    out, rs, acc = sg.select_per_tile(1.5 * co[:, :nb], co, c2, n2, ref, one, z, noisy, one, z,
                                      spec)
    assert not acc.any() and np.array_equal(out, co)


def test_stamp_snr_is_above_the_border_median():
    """On a bright sky every pixel has ref/sqrt(var) far above the threshold;
    only peaks standing snr_min sigmas above their stamp's border median are
    kept, and non-positive maxima are never candidates."""
    H, W = 50, 60
    ref = np.full((H, W), 1000.0)
    var = np.full((H, W), 100.0)
    ref[20, 20] = 1150.0                         # 15 sigma above the border
    ref[30, 40] = 1050.0                         # 5 sigma: rejected
    ref[12, 45] = 1100.0                         # exactly 10 sigma: kept (>=)
    z = np.zeros((H, W), np.uint8)
    cs = sg.select_stamps(ref, var, z, z, 1, 1, r=5, S=8, snr_min=10.0)
    assert cs == [[(20, 20), (12, 45)]]
    neg = -ref
    assert sg.select_stamps(neg, var, z, z, 1, 1, r=5, S=8, snr_min=1.0) == [[]]
    # a peak 10 sigma above its dark surroundings but below the tile's sky
    # (the median of the unmasked tile) is not a candidate
    low = ref.copy()
    low[25:45, 5:25] = 500.0
    low[35, 15] = 600.0
    assert sg.select_stamps(low, var, z, z, 1, 1, r=5, S=8, snr_min=10.0) == [[(20, 20), (12, 45)]]
    # masked pixels do not enter the sky: with only the dark region unmasked
    # the sky is 500 and its peak (whose stamp lies in that region) is kept
    m = np.ones((H, W), np.uint8)
    m[25:45, 5:25] = 0
    got = sg.select_stamps(low, var, m, z, 1, 1, r=5, S=8, snr_min=10.0)
    assert got == [[(35, 15)]]
    st = np.arange(36.0).reshape(6, 6)
    b = np.r_[st[0], st[-1], st[1:-1, 0], st[1:-1, -1]]
    assert sg.border_median(st) == np.median(b) == 17.5        # even count: middle pair
    # the peak at exactly 10 sigma is a near-tie of the border test; the sky
    # test (1100 - 1000)/10 = 10 is one too; nothing else is within 1e-6
    cs, near = sg.select_stamps(ref, var, z, z, 1, 1, r=5, S=8, snr_min=10.0, tie_tol=1e-6)
    assert cs == [[(20, 20), (12, 45)]] and near == [2]
