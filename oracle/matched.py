"""FP64 oracle of the matched-filter coadd (TEST INFRASTRUCTURE ONLY).

The paper coadds its sky tiles for point-source detection with a per-image
matched filter, the optimal method for background-limited images of Zackay &
Ofek (2017) (Deep Coaddition in Sky Segments).  Written out for registered
images j with per-pixel variance maps: each background-subtracted image
M_j = cal_j - bg_j is divided by its variance and cross-correlated with its
own PSF P_j (unit sum, half-width r), scaled by its flux zero point F_j, and
the images are summed:

    S(q)   = sum_j F_j   sum_u P_j(u)   M_j(q + u) / V_j(q + u)
    Var(q) = sum_j F_j^2 sum_u P_j(u)^2            / V_j(q + u)

over the pixels q + u inside the image whose mask is 0 and whose variance is
positive.  Var is the variance of S for independent pixel noise, and for a
point source of flux f at q, E[S(q)] = f Var(q): the flux estimate is
S/Var, its error Var^-1/2 and the detection SNR S/sqrt(Var) (0 where Var =
0).  For one image with F = 1 these are the PSF-weighted flux, its error and
the ratio of the two of the detection step.  u = (du, dv) indexes the PSF
stamp P[dv + r][du + r].
"""
from __future__ import annotations

import numpy as np


def matched_coadd(cals, vars_, masks, bgs, psfs, scales):
    """(S, Var, SNR) as float64 [H][W].  bgs: per image a background map
    ([H][W]) or None (images already background-subtracted)."""
    cals = [np.asarray(c, np.float64) for c in cals]
    H, W = cals[0].shape
    S = np.zeros((H, W))
    Var = np.zeros((H, W))
    for cal, var, msk, bg, P, F in zip(cals, vars_, masks, bgs, psfs, scales):
        var = np.asarray(var, np.float64)
        P = np.asarray(P, np.float64)
        r = P.shape[0] // 2
        M = cal - (0.0 if bg is None else np.asarray(bg, np.float64))
        ok = (np.asarray(msk) == 0) & (var > 0)
        a = np.zeros((H + 2 * r, W + 2 * r))        # M / V, zero off the image and where masked
        b = np.zeros((H + 2 * r, W + 2 * r))        # 1 / V likewise
        with np.errstate(all="ignore"):
            a[r:r + H, r:r + W] = np.where(ok, M / var, 0.0)
            b[r:r + H, r:r + W] = np.where(ok, 1.0 / var, 0.0)
        for dv in range(-r, r + 1):
            for du in range(-r, r + 1):
                p = P[dv + r, du + r]
                S += F * p * a[r + dv:r + dv + H, r + du:r + du + W]
                Var += F * F * p * p * b[r + dv:r + dv + H, r + du:r + du + W]
    snr = np.zeros((H, W))
    pos = Var > 0
    snr[pos] = S[pos] / np.sqrt(Var[pos])
    return S, Var, snr
