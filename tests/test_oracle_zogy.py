"""Pins of the ZOGY oracle: identical images give D = 0; D is white with
unit variance on pure noise; P_D has unit sum; a point source in the new
image is recovered in flux and position; with a noise-free delta-PSF
reference the proper difference is the classical difference (new minus the
reference convolved with the new PSF) over sigma_n."""
import numpy as np
import pytest

from oracle import zogy
from paper_2207_14304_amd import synth

L = 128


def _psf(r, fwhm):
    P = synth.psf_image(r, fwhm)
    return P / P.sum()                 # unit sum (the stamp truncates the Moffat wings)


def test_identical_images_subtract_to_zero():
    rng = np.random.default_rng(0)
    img = rng.uniform(0, 100, (L, L))
    P = _psf(5, 2.5)
    z = np.zeros((L, L), np.uint8)
    D, snr, flux, FD, pd2, m = zogy.zogy_tile(img, img, z, z, P, P, 1.0, 1.0, 3.0, 3.0)
    assert np.abs(D).max() < 1e-12 and np.abs(snr).max() < 1e-10


def test_pure_noise_is_white_and_unit():
    rng = np.random.default_rng(1)
    Pn, Pr = _psf(6, 3.0), _psf(6, 2.0)
    sn, sr = 7.0, 4.0
    vals, acs = [], []
    for _ in range(8):
        N = rng.standard_normal((L, L)) * sn
        R = rng.standard_normal((L, L)) * sr
        z = np.zeros((L, L), np.uint8)
        D, snr, *_ = zogy.zogy_tile(N, R, z, z, Pn, Pr, 1.1, 0.9, sn, sr)
        vals.append(D[8:-8, 8:-8].ravel())
        acs.append(np.mean(D[8:-8, 8:-9] * D[8:-8, 9:-8]))        # lag-1 autocorrelation
    v = np.concatenate(vals)
    assert abs(v.std() - 1.0) < 0.01 and abs(v.mean()) < 0.01
    assert abs(np.mean(acs)) < 0.01


def test_point_source_flux_and_unit_sum_psf():
    Pn, Pr = _psf(6, 3.0), _psf(6, 2.0)
    Fn, Fr, sn, sr = 1.2, 0.8, 5.0, 3.0
    N = np.zeros((L, L))
    N[60 - 6:60 + 7, 70 - 6:70 + 7] = Fn * 2500.0 * Pn
    R = np.zeros((L, L))
    z = np.zeros((L, L), np.uint8)
    D, snr, flux, FD, pd2, m = zogy.zogy_tile(N, R, z, z, Pn, Pr, Fn, Fr, sn, sr)
    assert FD == pytest.approx(Fn * Fr / np.sqrt(sn * sn * Fr * Fr + sr * sr * Fn * Fn), rel=1e-15)
    assert flux[60, 70] == pytest.approx(2500.0, rel=1e-10)
    assert np.unravel_index(np.argmax(snr), snr.shape) == (60, 70)
    assert snr[60, 70] == pytest.approx(FD * 2500.0 * np.sqrt(pd2), rel=1e-10)
    # P_D (the response of D to a unit point source, over F_D) has unit sum
    assert D.sum() / FD == pytest.approx(2500.0, rel=1e-9)


def test_delta_reference_reduces_to_classical_difference():
    rng = np.random.default_rng(3)
    Pn = _psf(5, 2.8)
    delta = np.zeros((11, 11))
    delta[5, 5] = 1.0
    sky = rng.uniform(0, 50, (L, L))
    N = np.real(np.fft.ifft2(np.fft.fft2(sky) * zogy._psf_hat(Pn, L))) * 1.3 + rng.standard_normal((L, L))
    z = np.zeros((L, L), np.uint8)
    D, *_ = zogy.zogy_tile(N, sky, z, z, Pn, delta, 1.3, 1.0, 2.0, 1e-30)
    classical = (N - 1.3 * np.real(np.fft.ifft2(np.fft.fft2(sky) * zogy._psf_hat(Pn, L)))) / 2.0
    assert np.allclose(D[6:-6, 6:-6], classical[6:-6, 6:-6], rtol=0, atol=1e-9)


def test_masks_and_edges():
    P = _psf(4, 2.0)
    z = np.zeros((L, L), np.uint8)
    mn = z.copy()
    mn[50, 50] = 1
    D, snr, flux, FD, pd2, m = zogy.zogy_tile(np.ones((L, L)), np.ones((L, L)), mn, z, P, P, 1.0,
                                             1.0, 1.0, 1.0)
    assert np.all(m[:4] != 0) and np.all(m[:, -4:] != 0) and m[10, 10] == 0
    assert np.all(m[42:59, 42:59] != 0) and m[50, 59] == 0 and m[50, 58] != 0
    assert np.all(D[m != 0] == 0)
