"""Pins of the background-map and source-detection oracle (closed forms):
constant and planar fields, stars in a minority of a cell's pixels, a
masked cell filled from its neighbours, a single outlying cell removed by
the 3 x 3 median, and sources of known flux and centroid."""
import numpy as np
import pytest

from oracle import background as bk
from paper_2207_14304_amd import synth


def test_cells_cover_the_frame():
    assert bk.cell_bounds(130, 64) == [(0, 64), (64, 128), (128, 130)]
    assert bk.cell_bounds(128, 64) == [(0, 64), (64, 128)]


def test_constant_field_with_masked_outliers():
    H, W = 150, 230                            # ragged last cells
    cal = np.full((H, W), 812.5)
    mask = np.zeros((H, W), np.uint8)
    rng = np.random.default_rng(0)
    hot = rng.random((H, W)) < 0.02
    cal[hot] = 60000.0
    mask[hot] = 1
    lev, grid, bgm = bk.background(cal, mask, 64)
    assert lev.shape == (3, 4)
    assert np.all(lev == 812.5) and np.all(grid == 812.5) and np.all(bgm == 812.5)


def test_planar_field_is_reproduced_between_interior_centres():
    H, W, box = 384, 448, 64                    # 6 x 7 whole cells
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    plane = 700.0 + 0.31 * x - 0.17 * y
    lev, grid, bgm = bk.background(plane, np.zeros((H, W), np.uint8), box)
    cx = np.arange(7) * box + (box - 1) / 2.0
    cy = np.arange(6) * box + (box - 1) / 2.0
    # a cell's median is the plane at its centre (symmetric values)
    assert np.allclose(lev, 700.0 + 0.31 * cx[None, :] - 0.17 * cy[:, None], rtol=0, atol=1e-9)
    # the 3 x 3 median of a planar grid is its centre at interior cells
    assert np.allclose(grid[1:-1, 1:-1], lev[1:-1, 1:-1], rtol=0, atol=1e-9)
    # bilinear interpolation reproduces the plane where all four nodes are interior cells
    sl = (slice(int(cy[1]) + 1, int(cy[-2])), slice(int(cx[1]) + 1, int(cx[-2])))
    assert np.allclose(bgm[sl], plane[sl], rtol=0, atol=1e-9)


def test_stars_in_a_minority_of_pixels_leave_the_level():
    H = W = 128
    cal = np.full((H, W), 800.0)
    P = synth.psf_image(7, 2.6)
    for (y, x) in ((20, 20), (30, 90), (100, 40), (90, 100)):
        cal[y - 7:y + 8, x - 7:x + 8] += 5e4 * P
    lev, grid, bgm = bk.background(cal, np.zeros((H, W), np.uint8), 64)
    assert np.all(lev == 800.0) and np.all(bgm == 800.0)


def test_masked_cell_and_outlying_cell():
    H, W, box = 320, 320, 64                    # 5 x 5 cells
    rng = np.random.default_rng(3)
    cal = 1000.0 + rng.standard_normal((H, W))
    mask = np.zeros((H, W), np.uint8)
    mask[128:192, 128:192] = 2                  # centre cell fully masked: no level
    cal[0:64, 256:320] += 500.0                 # corner cell far above its neighbours
    lev, grid, _ = bk.background(cal, mask, box)
    assert np.isnan(lev[2, 2])
    nb = np.delete(lev[1:4, 1:4].ravel(), 4)    # the eight present neighbours
    assert grid[2, 2] == np.median(nb)
    assert lev[0, 4] > 1400 and abs(grid[0, 4] - 1000.0) < 1.0
    # the map is the bilinear interpolation of the grid (spot check one pixel)
    g = np.arange(25.0).reshape(5, 5)
    m = bk.background_map(g, W, H, box)
    y, x = 100, 200                             # between centres 95.5/159.5 and 159.5/223.5
    ty, tx = (y - 95.5) / 64, (x - 159.5) / 64
    want = ((1 - ty) * ((1 - tx) * g[1, 2] + tx * g[1, 3]) + ty * ((1 - tx) * g[2, 2] + tx * g[2, 3]))
    assert m[y, x] == pytest.approx(want, rel=1e-14)
    assert m[0, 0] == g[0, 0] and m[-1, -1] == g[-1, -1]


def test_sources_flux_and_centroid():
    H, W = 160, 200
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    bgm = 600.0 + 0.2 * x + 0.1 * y
    cal = bgm.copy()
    var = np.full((H, W), 650.0)
    mask = np.zeros((H, W), np.uint8)
    P = synth.psf_image(5, 2.4)
    cal[60 - 5:60 + 6, 80 - 5:80 + 6] += 4321.0 * P        # symmetric: centroid at the pixel
    cal[120, 150] += 900.0                                   # two equal pixels: centroid halfway
    cal[120, 151] += 900.0
    snr, det, src = bk.detect_sources(cal, var, mask, bgm, 5.0, P)
    assert [(s["x"], s["y"]) for s in src] == [(80, 60), (150, 120)]
    a, b = src
    assert a["flux"] == pytest.approx(4321.0, rel=1e-12)
    assert a["flux_err"] == pytest.approx(np.sqrt(650.0 / (P * P).sum()), rel=1e-12)
    assert a["xc"] == pytest.approx(80.0, abs=1e-12) and a["yc"] == pytest.approx(60.0, abs=1e-12)
    assert b["xc"] == pytest.approx(150.5, abs=1e-12) and b["yc"] == pytest.approx(120.0, abs=1e-12)
    assert a["snr"] == pytest.approx(4321.0 * P[5, 5] / np.sqrt(650.0), rel=1e-12)
