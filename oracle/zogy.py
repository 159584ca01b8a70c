"""FP64 oracle of ZOGY image subtraction (TEST INFRASTRUCTURE ONLY).

The paper's second subtraction algorithm, for its 30-second cadence and deep
coadds, is that of Zackay, Ofek & Gal-Yam (2016, "ZOGY") (Transient Alerts;
Fig. 4; Table 2, 1400 ms per tile on one CPU core).  Written out from that
paper for one square tile of side L, in the Fourier domain of the tile
(hats; the transform treats the tile as periodic).  Inputs: the new image N
and the reference R, background-subtracted and registered, their PSFs P_n,
P_r (unit sum, centred), flux zero points F_n, F_r and background noise
sigmas s_n, s_r:

    den^2   = s_n^2 F_r^2 |P_r^|^2 + s_r^2 F_n^2 |P_n^|^2
    D^      = (F_r P_r^ N^ - F_n P_n^ R^) / den          (the proper difference)
    F_D     = F_n F_r / sqrt(s_n^2 F_r^2 + s_r^2 F_n^2)
    P_D^    = F_r F_n P_r^ P_n^ / (F_D den)              (its PSF, unit sum)
    S^      = D^ conj(P_D^)                                (matched filter)

D has white noise of unit variance when the images' noise is white with the
given sigmas; a point source of flux f at q gives D = F_D f P_D(x - q), so
S(q) = F_D f sum P_D^2 + noise of variance sum P_D^2.  The detection map is
SNR = S / sqrt(sum P_D^2) and the flux estimate S / (F_D sum P_D^2).

Readings (the paper gives none of these): the tile is square with a
power-of-two side; masked pixels enter N and R as 0; outputs within the PSF
half-width r of the tile border, or within 2r of a masked pixel (the support
of P_D * P_D), are flagged EDGE/FOOT and set to 0; PSF stamps are placed with
their centre at the origin of the periodic tile.
"""
from __future__ import annotations

import numpy as np

from .core import EDGE, FOOT


def _psf_hat(P, L):
    P = np.asarray(P, np.float64)
    r = P.shape[0] // 2
    big = np.zeros((L, L))
    for dv in range(-r, r + 1):
        for du in range(-r, r + 1):
            big[dv % L, du % L] += P[dv + r, du + r]
    return np.fft.fft2(big)


def zogy_tile(N, R, mask_n, mask_r, Pn, Pr, Fn, Fr, sn, sr):
    """(D, SNR, flux, F_D, sum P_D^2, out_mask) for one L x L tile."""
    N = np.asarray(N, np.float64)
    R = np.asarray(R, np.float64)
    L = N.shape[0]
    bad = (np.asarray(mask_n) != 0) | (np.asarray(mask_r) != 0)
    Nh = np.fft.fft2(np.where(bad, 0.0, N))
    Rh = np.fft.fft2(np.where(bad, 0.0, R))
    Pnh, Prh = _psf_hat(Pn, L), _psf_hat(Pr, L)
    den = np.sqrt(sn * sn * Fr * Fr * np.abs(Prh) ** 2 + sr * sr * Fn * Fn * np.abs(Pnh) ** 2)
    Dh = (Fr * Prh * Nh - Fn * Pnh * Rh) / den
    FD = Fn * Fr / np.sqrt(sn * sn * Fr * Fr + sr * sr * Fn * Fn)
    PDh = Fr * Fn * Prh * Pnh / (FD * den)
    D = np.real(np.fft.ifft2(Dh))
    S = np.real(np.fft.ifft2(Dh * np.conj(PDh)))
    pd2 = float(np.sum(np.abs(PDh) ** 2) / (L * L))          # Parseval: sum P_D^2
    snr = S / np.sqrt(pd2)
    flux = S / (FD * pd2)
    r = max(np.asarray(Pn).shape[0], np.asarray(Pr).shape[0]) // 2
    out = np.zeros((L, L), np.uint8)
    out[:r, :] = out[-r:, :] = EDGE
    out[:, :r] = EDGE
    out[:, -r:] = EDGE
    if bad.any():
        ys, xs = np.nonzero(bad)
        near = np.zeros((L, L), bool)
        for y, x in zip(ys, xs):
            near[max(y - 2 * r, 0):y + 2 * r + 1, max(x - 2 * r, 0):x + 2 * r + 1] = True
        out[near] |= FOOT
    z = out != 0
    return (np.where(z, 0.0, D), np.where(z, 0.0, snr), np.where(z, 0.0, flux), FD, pd2, out)
