"""FP64 oracle of the background map and full-frame source detection
(TEST INFRASTRUCTURE ONLY).

The paper's GPU pipeline computes a median-filtered background map and
detects sources on every full frame before astrometry (Pipeline
Implementation; Table 2, 1.7 ms and 6.1 ms on its GPU); the compute nodes
keep background and noise maps beside the calibration frames (Compute
Nodes).  It prints no formulas, so each step here is a stated reading:

* background cells: the frame is cut into box x box cells from the origin
  (the last row and column of cells may be narrower); a cell's level is the
  median of its unmasked calibrated values (mask == 0; an even count takes
  the mean of the middle two); a cell without unmasked pixels has none;
* median filter: each cell's map value is the median of the levels present
  in its 3 x 3 neighbourhood of cells (within the grid); 0 when none is;
* map: bilinear interpolation between cell centres ((x0 + x1 - 1)/2 of a
  cell spanning [x0, x1)), held constant beyond the first and last centres;
* sources: on D = cal - background with V = var (the calibration's noise
  map) and the calibration mask, the detection of the difference image
  (SNR = D/sqrt(V), threshold, raster-ordered local maxima, PSF-weighted
  flux); each source also gets the centroid of max(D, 0) over its unmasked
  in-image 3 x 3 neighbourhood (NaN when that sum is not positive).
"""
from __future__ import annotations

import numpy as np

from . import core

SRC_DTYPE = np.dtype([("x", np.int32), ("y", np.int32), ("xc", np.float64), ("yc", np.float64),
                      ("snr", np.float64), ("flux", np.float64), ("flux_err", np.float64)])


def cell_bounds(n, box):
    """[(start, stop)] of the cells along an axis of n pixels."""
    return [(s, min(s + box, n)) for s in range(0, n, box)]


def cell_levels(cal, mask, box):
    """Median of the unmasked values of every cell, [gy][gx]; NaN where a
    cell has no unmasked pixel."""
    cal = np.asarray(cal, np.float64)
    mask = np.asarray(mask)
    H, W = cal.shape
    bx, by = cell_bounds(W, box), cell_bounds(H, box)
    out = np.full((len(by), len(bx)), np.nan)
    for j, (y0, y1) in enumerate(by):
        for i, (x0, x1) in enumerate(bx):
            v = cal[y0:y1, x0:x1][mask[y0:y1, x0:x1] == 0]
            if v.size:
                out[j, i] = np.median(v)
    return out


def median_filter3(levels):
    """3 x 3 median over the levels present (non-NaN) around each cell."""
    gy, gx = levels.shape
    out = np.zeros_like(levels)
    for j in range(gy):
        for i in range(gx):
            nb = levels[max(j - 1, 0):j + 2, max(i - 1, 0):i + 2].ravel()
            nb = nb[~np.isnan(nb)]
            out[j, i] = np.median(nb) if nb.size else 0.0
    return out


def _axis_weights(n, box):
    """Per pixel of an axis: (index of the left node, weight of the right)."""
    cen = np.array([(a + b - 1) / 2.0 for (a, b) in cell_bounds(n, box)])
    x = np.arange(n, dtype=np.float64)
    i = np.searchsorted(cen, x, side="right") - 1            # last centre <= x
    i = np.clip(i, 0, len(cen) - 1)
    t = np.zeros(n)
    inner = (x >= cen[0]) & (i < len(cen) - 1)
    t[inner] = (x[inner] - cen[i[inner]]) / (cen[i[inner] + 1] - cen[i[inner]])
    return i, t


def background_map(grid, W, H, box):
    """Bilinear interpolation of the filtered grid to every pixel."""
    grid = np.asarray(grid, np.float64)
    ix, tx = _axis_weights(W, box)
    iy, ty = _axis_weights(H, box)
    ix1 = np.minimum(ix + 1, grid.shape[1] - 1)
    iy1 = np.minimum(iy + 1, grid.shape[0] - 1)
    g00 = grid[np.ix_(iy, ix)]
    g01 = grid[np.ix_(iy, ix1)]
    g10 = grid[np.ix_(iy1, ix)]
    g11 = grid[np.ix_(iy1, ix1)]
    tx = tx[None, :]
    ty = ty[:, None]
    top = g00 + tx * (g01 - g00)
    bot = g10 + tx * (g11 - g10)
    return top + ty * (bot - top)


def background(cal, mask, box=64):
    """(raw cell levels, filtered grid, full-resolution map)."""
    lev = cell_levels(cal, mask, box)
    grid = median_filter3(lev)
    H, W = np.shape(cal)
    return lev, grid, background_map(grid, W, H, box)


def detect_sources(cal, var, mask, bg_map, threshold, psf):
    """Sources on the background-subtracted frame.  Returns (snr, det_mask,
    sources) with sources sorted by raster index (SRC_DTYPE)."""
    D = np.asarray(cal, np.float64) - np.asarray(bg_map, np.float64)
    V = np.asarray(var, np.float64)
    M = np.asarray(mask)
    snr, det, c = core.detect(D, V, M, threshold, psf)
    H, W = D.shape
    good = (M == 0) & (V > 0)
    out = np.zeros(c.size, SRC_DTYPE)
    for n, cand in enumerate(c):
        x, y = int(cand["x"]), int(cand["y"])
        s = sx = sy = 0.0
        for v in (-1, 0, 1):
            for u in (-1, 0, 1):
                xx, yy = x + u, y + v
                if 0 <= xx < W and 0 <= yy < H and good[yy, xx]:
                    d = max(D[yy, xx], 0.0)
                    s += d
                    sx += u * d
                    sy += v * d
        xc = x + sx / s if s > 0 else np.nan
        yc = y + sy / s if s > 0 else np.nan
        out[n] = (x, y, xc, yc, cand["snr"], cand["flux"], cand["flux_err"])
    return snr, det, out
