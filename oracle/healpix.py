"""FP64 oracle of the resampling of a calibrated frame into HEALPix-aligned
segment images (TEST INFRASTRUCTURE ONLY).

The paper reprojects every full frame into equal-area sky tiles of the
HEALPix pixelization (Gorski et al. 2005) at NSIDE = 256, 13.7 arcmin
across, on the GPU (Image Segmentation; Pipeline Implementation; Table 2,
3.2 ms).  It names neither the segment pixel grid nor the interpolation, so
these are readings:

* sky geometry: the HEALPix projection of the sphere onto the plane
  (x_s, y_s) (Gorski et al. 2005; Calabretta & Roukema 2007): with
  z = cos(theta),
    |z| <= 2/3:  x_s = phi,  y_s = (3 pi / 8) z;
    |z| >  2/3:  sigma = sqrt(3 (1 - |z|)),  x_s = phi_c + (phi - phi_c) sigma,
                 y_s = sign(z) (pi / 4) (2 - sigma),
  phi_c = pi/4 + k pi/2 the centre of phi's quadrant.  The twelve base
  pixels are the diamonds of half-diagonal pi/4 centred at
  (pi/4 + f pi/2, pi/4) for f = 0..3 (their north corners are the pole),
  ((f - 4) pi/2, 0) for f = 4..7 (x_s periodic in 2 pi) and
  (pi/4 + (f - 8) pi/2, -pi/4) for f = 8..11;
* face coordinates: (a, b) in [0, 1]^2 with x_s = x_c + (pi/4)(a - b) and
  y_s = y_c + (pi/4)(a + b - 1), so a runs from the diamond's south corner
  to its east corner and b from the south corner to its west corner;
* tiles and segments: tile (f, I, J) of NSIDE n covers a in [I/n, (I+1)/n),
  b in [J/n, (J+1)/n) of face f; its segment image has m x m pixels, pixel
  (p, q) (row q, column p) centred at a = (I m + p + 1/2)/(n m),
  b = (J m + q + 1/2)/(n m): the HEALPix pixels of NSIDE n m inside the
  tile;
* frame geometry: a gnomonic (TAN) world coordinate system with reference
  pixel (crpix1, crpix2), reference direction (ra0, dec0) and a 2 x 2
  matrix cd (degrees per pixel) from pixel offsets to standard coordinates
  (xi, eta) (Calabretta & Greisen 2002);
* values: bilinear interpolation of the calibrated frame at the segment
  pixel's frame position; the variance is sum w^2 var over the four
  neighbours (independent pixels); a segment pixel is NODATA where its
  position is not inside [0, W-1] x [0, H-1] or any of the four neighbours is
  masked (then value = variance = 0).
"""
from __future__ import annotations

import math

import numpy as np

from .core import NODATA

HP = math.pi / 2
QP = math.pi / 4


def face_centre(f):
    """(x_c, y_c) of base pixel f in the projection plane."""
    if f < 4:
        return QP + f * HP, QP
    if f < 8:
        return (f - 4) * HP, 0.0
    return QP + (f - 8) * HP, -QP


def face_to_plane(f, a, b):
    xc, yc = face_centre(f)
    return xc + QP * (np.asarray(a) - np.asarray(b)), yc + QP * (np.asarray(a) + np.asarray(b) - 1)


def plane_to_sphere(xs, ys):
    """Inverse HEALPix projection: (z, phi) with phi in [0, 2 pi)."""
    xs = np.mod(np.asarray(xs, np.float64), 2 * math.pi)
    ys = np.asarray(ys, np.float64)
    z = np.empty(np.broadcast(xs, ys).shape)
    phi = np.empty_like(z)
    eq = np.abs(ys) <= QP
    z[eq] = ys[eq] * 8.0 / (3.0 * math.pi)
    phi[eq] = xs[eq]
    po = ~eq
    sig = 2.0 - np.abs(ys[po]) / QP
    z[po] = np.sign(ys[po]) * (1.0 - sig * sig / 3.0)
    phic = QP + np.floor(xs[po] / HP) * HP
    with np.errstate(all="ignore"):
        phi[po] = np.where(sig > 0, phic + (xs[po] - phic) / np.where(sig > 0, sig, 1.0), phic)
    return z, np.mod(phi, 2 * math.pi)


def sphere_to_plane(z, phi):
    """Forward HEALPix projection of (z, phi)."""
    z = np.asarray(z, np.float64)
    phi = np.mod(np.asarray(phi, np.float64), 2 * math.pi)
    xs = np.empty(np.broadcast(z, phi).shape)
    ys = np.empty_like(xs)
    eq = np.abs(z) <= 2.0 / 3.0
    xs[eq] = phi[eq]
    ys[eq] = 3.0 * math.pi / 8.0 * z[eq]
    po = ~eq
    sig = np.sqrt(3.0 * (1.0 - np.abs(z[po])))
    phic = QP + np.floor(phi[po] / HP) * HP
    xs[po] = phic + (phi[po] - phic) * sig
    ys[po] = np.sign(z[po]) * QP * (2.0 - sig)
    return xs, ys


def plane_to_face(xs, ys):
    """(face, a, b) of plane points (x_s in [0, 2 pi))."""
    xs = np.mod(np.asarray(xs, np.float64), 2 * math.pi)
    ys = np.asarray(ys, np.float64)
    face = np.full(xs.shape, -1)
    a = np.zeros(xs.shape)
    b = np.zeros(xs.shape)
    for f in range(12):
        xc, yc = face_centre(f)
        dx = np.mod(xs - xc + math.pi, 2 * math.pi) - math.pi      # periodic in x
        u, v = dx / QP, (ys - yc) / QP
        aa, bb = (1 + u + v) / 2, (1 - u + v) / 2
        inside = (aa >= 0) & (aa < 1) & (bb >= 0) & (bb < 1) & (face < 0)
        face[inside] = f
        a[inside] = aa[inside]
        b[inside] = bb[inside]
    return face, a, b


def radec_to_zphi(ra, dec):
    return np.sin(np.radians(dec)), np.radians(ra)


def zphi_to_radec(z, phi):
    return np.degrees(phi), np.degrees(np.arcsin(np.clip(z, -1, 1)))


class Wcs:
    """Gnomonic projection: pixel (x, y) <-> (ra, dec) in degrees."""

    def __init__(self, ra0, dec0, crpix1, crpix2, cd):
        self.ra0, self.dec0 = float(ra0), float(dec0)
        self.crpix = (float(crpix1), float(crpix2))
        self.cd = np.asarray(cd, np.float64).reshape(2, 2)
        self.cdi = np.linalg.inv(self.cd)

    def sky_to_pixel(self, ra, dec):
        a0, d0 = math.radians(self.ra0), math.radians(self.dec0)
        a, d = np.radians(ra), np.radians(dec)
        den = np.sin(d) * math.sin(d0) + np.cos(d) * math.cos(d0) * np.cos(a - a0)
        xi = np.degrees(np.cos(d) * np.sin(a - a0) / den)
        eta = np.degrees((np.sin(d) * math.cos(d0) - np.cos(d) * math.sin(d0) * np.cos(a - a0)) / den)
        x = self.cdi[0, 0] * xi + self.cdi[0, 1] * eta + self.crpix[0]
        y = self.cdi[1, 0] * xi + self.cdi[1, 1] * eta + self.crpix[1]
        return x, y, den

    def pixel_to_sky(self, x, y):
        dx, dy = np.asarray(x, np.float64) - self.crpix[0], np.asarray(y, np.float64) - self.crpix[1]
        xi = np.radians(self.cd[0, 0] * dx + self.cd[0, 1] * dy)
        eta = np.radians(self.cd[1, 0] * dx + self.cd[1, 1] * dy)
        a0, d0 = math.radians(self.ra0), math.radians(self.dec0)
        rho = np.hypot(xi, eta)
        c = np.arctan(rho)
        with np.errstate(all="ignore"):
            s = np.where(rho > 0, eta * np.sin(c) / np.where(rho > 0, rho, 1.0), 0.0)
        dec = np.arcsin(np.cos(c) * math.sin(d0) + s * math.cos(d0))
        ra = a0 + np.arctan2(xi * np.sin(c), rho * math.cos(d0) * np.cos(c) - eta * math.sin(d0) * np.sin(c))
        return np.mod(np.degrees(ra), 360.0), np.degrees(dec)


def segment_positions(wcs, tile, nside, m):
    """Frame pixel positions (x, y) [m][m] of the segment pixels of tile
    (f, I, J) at NSIDE nside with m x m pixels; den <= 0 marks directions on
    the far side of the tangent plane."""
    f, I, J = tile
    p = np.arange(m)
    a = (I * m + p[None, :] + 0.5) / (nside * m)
    b = (J * m + p[:, None] + 0.5) / (nside * m)
    xs, ys = face_to_plane(f, a, b)
    z, phi = plane_to_sphere(xs, ys)
    ra, dec = zphi_to_radec(z, phi)
    return wcs.sky_to_pixel(ra, dec)


def resample(cal, var, mask, wcs, tiles, nside, m):
    """Segment images (value, variance, mask), each [n_tiles][m][m]."""
    cal = np.asarray(cal, np.float64)
    var = np.asarray(var, np.float64)
    mask = np.asarray(mask)
    H, W = cal.shape
    out = np.zeros((len(tiles), m, m))
    outv = np.zeros((len(tiles), m, m))
    outm = np.zeros((len(tiles), m, m), np.uint8)
    for t, tile in enumerate(tiles):
        x, y, den = segment_positions(wcs, tile, nside, m)
        ok = (den > 0) & (x >= 0) & (x <= W - 1) & (y >= 0) & (y <= H - 1)
        x0 = np.clip(np.floor(x), 0, max(W - 2, 0)).astype(np.int64)
        y0 = np.clip(np.floor(y), 0, max(H - 2, 0)).astype(np.int64)
        x1 = np.minimum(x0 + 1, W - 1)
        y1 = np.minimum(y0 + 1, H - 1)
        fx = np.where(ok, x - x0, 0.0)
        fy = np.where(ok, y - y0, 0.0)
        w = [(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy]
        nb = [(y0, x0), (y0, x1), (y1, x0), (y1, x1)]
        bad = np.zeros((m, m), bool)
        for (yy, xx) in nb:
            bad |= mask[yy, xx] != 0
        val = sum(wi * cal[yy, xx] for wi, (yy, xx) in zip(w, nb))
        vv = sum(wi * wi * var[yy, xx] for wi, (yy, xx) in zip(w, nb))
        good = ok & ~bad
        out[t] = np.where(good, val, 0.0)
        outv[t] = np.where(good, vv, 0.0)
        outm[t] = np.where(good, 0, NODATA)
    return out, outv, outm


def tiles_of_frame(wcs, W, H, nside, step=32):
    """The tiles (f, I, J) at NSIDE nside that frame pixels fall in, sampled
    every `step` pixels and along the border, sorted."""
    xs = np.r_[np.arange(0, W, step), W - 1]
    ys = np.r_[np.arange(0, H, step), H - 1]
    X, Y = np.meshgrid(xs, ys)
    ra, dec = wcs.pixel_to_sky(X.ravel(), Y.ravel())
    z, phi = radec_to_zphi(ra, dec)
    f, a, b = plane_to_face(*sphere_to_plane(z, phi))
    I = np.minimum((a * nside).astype(np.int64), nside - 1)
    J = np.minimum((b * nside).astype(np.int64), nside - 1)
    return sorted(set(zip(f.tolist(), I.tolist(), J.tolist())))
