"""Pins of the matched-filter coadd oracle: a point source's flux and SNR in
closed form, N identical exposures (SNR grows as sqrt(N), flux unchanged),
unit-variance SNR on pure noise, and equality with the detection step's
PSF-weighted flux for one image."""
import math

import numpy as np
import pytest

import oracle
from oracle import matched
from paper_2207_14304_amd import synth


def test_point_source_closed_form():
    H, W, r = 60, 70, 5
    P = synth.psf_image(r, 2.4)
    M = np.zeros((H, W))
    M[30 - r:30 + r + 1, 40 - r:40 + r + 1] = 777.0 * P
    var = np.full((H, W), 400.0)
    z = np.zeros((H, W), np.uint8)
    S, Var, snr = matched.matched_coadd([M], [var], [z], [None], [P], [1.0])
    q = (P * P).sum() / 400.0
    assert Var[30, 40] == pytest.approx(q, rel=1e-13)
    assert S[30, 40] / Var[30, 40] == pytest.approx(777.0, rel=1e-12)
    assert snr[30, 40] == pytest.approx(777.0 * math.sqrt(q), rel=1e-12)
    # the score peaks at the source (the matched filter's maximum)
    assert np.unravel_index(np.argmax(S), S.shape) == (30, 40)


def test_identical_exposures_and_zero_points():
    H, W, r = 50, 50, 4
    P = synth.psf_image(r, 2.0)
    rng = np.random.default_rng(1)
    M = rng.standard_normal((H, W)) * 10.0
    M[25 - r:25 + r + 1, 20 - r:20 + r + 1] += 500.0 * P
    var = np.full((H, W), 100.0)
    z = np.zeros((H, W), np.uint8)
    S1, V1, n1 = matched.matched_coadd([M], [var], [z], [None], [P], [1.0])
    S4, V4, n4 = matched.matched_coadd([M] * 4, [var] * 4, [z] * 4, [None] * 4, [P] * 4, [1.0] * 4)
    assert np.allclose(S4, 4 * S1, rtol=1e-12) and np.allclose(V4, 4 * V1, rtol=1e-12)
    assert np.allclose(n4, 2 * n1, rtol=1e-12, atol=1e-12)
    # an image twice as transparent (F = 2) recorded twice the counts: the
    # same flux estimate S/Var in the units of F = 1
    S2, V2, _ = matched.matched_coadd([2 * M], [4 * var], [z], [None], [P], [2.0])
    assert np.allclose(S2 / V2, S1 / V1, rtol=1e-12)


def test_pure_noise_snr_is_standard_normal():
    rng = np.random.default_rng(2)
    H, W, r = 700, 700, 3
    P = synth.psf_image(r, 1.8)
    imgs, vars_ = [], []
    for j in range(3):
        v = rng.uniform(50, 150, (H, W))
        vars_.append(v)
        imgs.append(rng.standard_normal((H, W)) * np.sqrt(v))
    z = np.zeros((H, W), np.uint8)
    _, _, snr = matched.matched_coadd(imgs, vars_, [z] * 3, [None] * 3,
                                      [synth.psf_image(r, 1.8 + 0.4 * j) for j in range(3)],
                                      [1.0, 0.8, 1.2])
    s = snr[r:-r, r:-r]
    assert abs(s.mean()) <= 0.01 and abs(s.std() - 1.0) <= 0.01


def test_one_image_equals_the_detection_psf_flux():
    H, W, r = 80, 90, 5
    rng = np.random.default_rng(4)
    P = synth.psf_image(r, 2.6)
    D = rng.standard_normal((H, W)) * 8.0
    D[40 - r:40 + r + 1, 45 - r:45 + r + 1] += 3000.0 * P
    V = rng.uniform(50, 80, (H, W))
    msk = np.zeros((H, W), np.uint8)
    msk[38, 44] = oracle.FOOT                  # a masked pixel inside the window
    bg = np.full((H, W), 5.0)
    S, Var, snr = matched.matched_coadd([D + bg], [V], [msk], [bg], [P], [1.0])
    _, _, c = oracle.detect(D, V, msk, 5.0, P)
    top = c[np.argmax(c["flux"])]
    x, y = top["x"], top["y"]
    assert S[y, x] / Var[y, x] == pytest.approx(top["flux"], rel=1e-12)
    assert Var[y, x] ** -0.5 == pytest.approx(top["flux_err"], rel=1e-12)
