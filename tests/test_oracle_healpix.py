"""Pins of the HEALPix segment resampling oracle: the projection's zones and
base-pixel centres, forward/inverse round trips, equal pixel areas (the
solid angle of a face-coordinate cell by the projection's Jacobian is
4 pi / (12 n^2) everywhere), the gnomonic frame geometry, and exact
reproduction of planar frames by the bilinear resampling."""
import math

import numpy as np
import pytest

from oracle import healpix as hp
from oracle.core import NODATA


def test_base_pixel_centres():
    # north faces: z = 2/3 at phi = pi/4 + f pi/2; equatorial: z = 0 at f pi/2
    for f in range(12):
        xs, ys = hp.face_to_plane(f, 0.5, 0.5)
        z, phi = hp.plane_to_sphere(np.array([xs]), np.array([ys]))
        zc = 2.0 / 3.0 if f < 4 else (0.0 if f < 8 else -2.0 / 3.0)
        pc = (math.pi / 4 + (f % 4) * math.pi / 2) if (f < 4 or f >= 8) else (f - 4) * math.pi / 2
        assert z[0] == pytest.approx(zc, abs=1e-15) and phi[0] == pytest.approx(pc, abs=1e-15)
    # the north corner of a north face is the pole
    z, _ = hp.plane_to_sphere(*[np.array([v]) for v in hp.face_to_plane(2, 1.0, 1.0)])
    assert z[0] == pytest.approx(1.0, abs=1e-15)


def test_round_trips_and_faces_cover_the_sphere():
    rng = np.random.default_rng(0)
    z = rng.uniform(-1, 1, 200000)
    phi = rng.uniform(0, 2 * math.pi, 200000)
    f, a, b = hp.plane_to_face(*hp.sphere_to_plane(z, phi))
    assert np.all(f >= 0)
    # equal-area faces: each receives a twelfth of uniform directions
    counts = np.bincount(f, minlength=12) / f.size
    assert np.all(np.abs(counts - 1 / 12) < 4 * math.sqrt(1 / 12 / f.size))
    z2, phi2 = np.empty_like(z), np.empty_like(z)
    for k in range(12):
        s = f == k
        z2[s], phi2[s] = hp.plane_to_sphere(*hp.face_to_plane(k, a[s], b[s]))
    assert np.abs(z2 - z).max() < 1e-12
    dphi = np.abs(np.mod(phi2 - phi + math.pi, 2 * math.pi) - math.pi)
    assert np.max(dphi * np.sqrt(1 - z * z)) < 1e-12


@pytest.mark.parametrize("face", [0, 5, 9])
def test_cells_have_equal_solid_angle(face):
    """d(solid angle) = dz dphi; the area of a face-coordinate cell of side
    1/n is 4 pi / (12 n^2) wherever it lies (numerical Jacobian)."""
    n = 64
    rng = np.random.default_rng(face)
    a = rng.uniform(0.05, 0.95, 500)
    b = rng.uniform(0.05, 0.95, 500)
    h = 1e-6

    def zp(aa, bb):
        return hp.plane_to_sphere(*hp.face_to_plane(face, aa, bb))

    za, pa = zp(a + h, b)
    zb, pb = zp(a - h, b)
    zc, pc = zp(a, b + h)
    zd, pd = zp(a, b - h)
    dza, dpa = (za - zb) / (2 * h), (pa - pb) / (2 * h)
    dzb, dpb = (zc - zd) / (2 * h), (pc - pd) / (2 * h)
    jac = np.abs(dza * dpb - dzb * dpa)
    assert np.allclose(jac / n ** 2, 4 * math.pi / (12 * n ** 2), rtol=1e-6)


def _wcs():
    s = 1.38 / 3600.0
    c, t = math.cos(0.3), math.sin(0.3)
    return hp.Wcs(83.6, 22.0, 4787.5, 3193.5, [[-s * c, s * t], [s * t, s * c]])


def test_gnomonic_round_trip_and_scale():
    w = _wcs()
    ra, dec = w.pixel_to_sky(np.array([4787.5]), np.array([3193.5]))
    assert ra[0] == pytest.approx(83.6, abs=1e-12) and dec[0] == pytest.approx(22.0, abs=1e-12)
    rng = np.random.default_rng(1)
    x, y = rng.uniform(0, 9576, 1000), rng.uniform(0, 6388, 1000)
    x2, y2, den = w.sky_to_pixel(*w.pixel_to_sky(x, y))
    assert np.all(den > 0) and np.abs(x2 - x).max() < 1e-7 and np.abs(y2 - y).max() < 1e-7
    # one pixel step near the reference point spans 1.38 arcsec
    r1, d1 = w.pixel_to_sky(np.array([4787.5, 4788.5]), np.array([3193.5, 3193.5]))
    d0r, d1r, da = math.radians(d1[0]), math.radians(d1[1]), math.radians(r1[1] - r1[0])
    hav = math.sin((d1r - d0r) / 2) ** 2 + math.cos(d0r) * math.cos(d1r) * math.sin(da / 2) ** 2
    sep = math.degrees(2 * math.asin(math.sqrt(hav)))          # haversine: exact for small angles
    assert sep * 3600 == pytest.approx(1.38, rel=1e-6)


def test_segment_pixels_are_the_fine_healpix_cells():
    """A segment pixel's sky position lies in its own tile and, at the fine
    NSIDE n m, in the cell (I m + p, J m + q)."""
    n, m = 256, 600
    tile = (4, 130, 117)
    w = hp.Wcs(0.0, 0.0, 0.0, 0.0, [[1e-4, 0], [0, 1e-4]])
    x, y, den = hp.segment_positions(w, tile, n, m)
    ra, dec = w.pixel_to_sky(x, y)
    f, a, b = hp.plane_to_face(*hp.sphere_to_plane(*hp.radec_to_zphi(ra, dec)))
    assert np.all(f == 4)
    p = np.arange(m)
    assert np.array_equal(np.floor(a * n * m).astype(int), np.broadcast_to(130 * m + p[None, :], (m, m)))
    assert np.array_equal(np.floor(b * n * m).astype(int), np.broadcast_to(117 * m + p[:, None], (m, m)))


def test_resampling_reproduces_planes_and_masks():
    W, H = 900, 700
    s = 1.38 / 3600.0
    w = hp.Wcs(10.0, 5.0, 449.5, 349.5, [[-s, 0.0], [0.0, s]])
    tiles = hp.tiles_of_frame(w, W, H, 256)
    assert 2 <= len(tiles) <= 12
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    cal = 500.0 + 0.25 * x - 0.125 * y
    var = np.full((H, W), 7.0)
    mask = np.zeros((H, W), np.uint8)
    mask[300, 400] = 1
    val, vv, mm = hp.resample(cal, var, mask, w, tiles, 256, 600)
    px, py = [], []
    for t in tiles:
        xx, yy, _ = hp.segment_positions(w, t, 256, 600)
        px.append(xx)
        py.append(yy)
    px, py = np.array(px), np.array(py)
    good = mm == 0
    assert good.sum() > 0.9 * W * H * (1.38 / (13.7 * 60 / 600)) ** 2
    assert np.allclose(val[good], (500.0 + 0.25 * px - 0.125 * py)[good], rtol=0, atol=1e-9)
    # variance: sum of squared bilinear weights times 7 (between 7/4 and 7)
    assert np.all((vv[good] >= 7.0 / 4 - 1e-12) & (vv[good] <= 7.0 + 1e-12))
    inside = (px >= 0) & (px <= W - 1) & (py >= 0) & (py <= H - 1)
    # NODATA: outside the frame, or the masked pixel among the four neighbours
    touches = np.isin(np.floor(px), [399, 400]) & np.isin(np.floor(py), [299, 300])
    assert np.array_equal(~good, ~inside | (inside & touches)) and touches.any()
    assert np.all(mm[~good] == NODATA) and np.all(val[~good] == 0)
