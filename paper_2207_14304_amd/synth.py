"""Seeded synthetic sCMOS frames for PSF-matched difference imaging.

This module only draws inputs: star fields, calibration masters, noise,
cosmic rays, transients and cutout tables.  It holds none of the arithmetic
of the reduction itself (calibration, coaddition, kernel fit, subtraction,
detection); both the HIP path and the CPU oracle consume what it returns.

Shapes follow the sensor described in the paper (Table 1 and the Image
Management section: IMX455, 61 MPix, 16-bit, 1.7 e- read noise).  The star
population, PSF and seeing follow the workloads the benchmark and tests use:

* positions uniform over the frame;
* fluxes with dN/dm proportional to 10^(0.3 m) between 1e2 and 1e6 e-, i.e.
  dN/df proportional to f^-1.75, drawn by inverting the CDF;
* Moffat PSF (beta = 3) sampled at pixel centres, truncated at 8 FWHM and
  renormalised to unit sum over the truncated disk;
* expected counts flat * (sky + scene), Poisson plus Gaussian read noise,
  ADU = counts / gain + dark, rounded half-to-even and clipped to 0..65535.

Every random stream comes from ``numpy.random.SeedSequence(seed).spawn``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

IMX455_W = 9576
IMX455_H = 6388
READ_NOISE_E = 1.7
SAT_ADU = 65535

# stream indices of SeedSequence(seed).spawn(N_STREAMS)
_S_STARS, _S_MASTERS, _S_TRANS, _S_CUT, _S_EXTRA = 0, 1, 2, 3, 4
_S_FRAME0 = 5            # frame i uses stream _S_FRAME0 + i (noise + cosmics)
N_STREAMS = 5 + 16


def moffat_alpha(fwhm: float, beta: float = 3.0) -> float:
    """Moffat core radius for a given FWHM."""
    return fwhm / (2.0 * math.sqrt(2.0 ** (1.0 / beta) - 1.0))


def draw_fluxes(rng: np.random.Generator, n: int, fmin: float = 1e2,
                fmax: float = 1e6) -> np.ndarray:
    """Power-law fluxes, dN/df ~ f^-1.75, by inverse CDF."""
    u = rng.random(n)
    a, b = fmax ** -0.75, fmin ** -0.75
    return (a + u * (b - a)) ** (-4.0 / 3.0)


def moffat_stamp(dx: np.ndarray, dy: np.ndarray, fwhm: float, beta: float = 3.0,
                 ellip: float = 0.0, theta: float = 0.0) -> np.ndarray:
    """Unnormalised Moffat profile at offsets (dx, dy) from the centre."""
    alpha = moffat_alpha(fwhm, beta)
    if ellip > 0.0:
        c, s = math.cos(theta), math.sin(theta)
        xr = c * dx + s * dy
        yr = (-s * dx + c * dy) / (1.0 - ellip)
        r2 = xr * xr + yr * yr
    else:
        r2 = dx * dx + dy * dy
    return (1.0 + r2 / (alpha * alpha)) ** (-beta)


def psf_image(half: int, fwhm: float, beta: float = 3.0, ellip: float = 0.0,
              theta: float = 0.0) -> np.ndarray:
    """Centred, unit-sum Moffat PSF on a (2*half+1)^2 grid, indexed [v+half][u+half].

    The disk truncation at 8 FWHM is applied before renormalising, exactly as
    for rendered stars, so a transient rendered with this PSF and the stamp
    passed to detection agree where the stamp covers it."""
    v, u = np.mgrid[-half:half + 1, -half:half + 1].astype(np.float64)
    p = moffat_stamp(u, v, fwhm, beta, ellip, theta)
    p[u * u + v * v > (8.0 * fwhm) ** 2] = 0.0
    full = _truncated_norm(fwhm, beta, ellip, theta)
    return p / full


def _truncated_norm(fwhm, beta, ellip, theta):
    rmax = 8.0 * fwhm
    rr = int(math.ceil(rmax))
    v, u = np.mgrid[-rr:rr + 1, -rr:rr + 1].astype(np.float64)
    p = moffat_stamp(u, v, fwhm, beta, ellip, theta)
    p[u * u + v * v > rmax * rmax] = 0.0
    return p.sum()


def render_scene(W: int, H: int, xs, ys, fluxes, fwhm_of_x, beta: float = 3.0,
                 ellip=None, theta=None) -> np.ndarray:
    """Sum of truncated unit-sum Moffat stars, float64 [H][W] (electrons).

    ``fwhm_of_x`` maps an array of star x positions to FWHMs (seeing that
    varies across the field).  Stars partly outside the frame lose the flux
    that falls outside."""
    img = np.zeros((H, W), np.float64)
    xs = np.asarray(xs, np.float64)
    ys = np.asarray(ys, np.float64)
    fluxes = np.asarray(fluxes, np.float64)
    fw = np.broadcast_to(np.asarray(fwhm_of_x(xs), np.float64), xs.shape)
    for i in range(xs.size):
        f = fw[i]
        e = 0.0 if ellip is None else float(ellip[i])
        t = 0.0 if theta is None else float(theta[i])
        rmax = 8.0 * f
        rr = int(math.ceil(rmax))
        xi, yi = int(round(xs[i])), int(round(ys[i]))
        x0, x1 = max(xi - rr, 0), min(xi + rr + 1, W)
        y0, y1 = max(yi - rr, 0), min(yi + rr + 1, H)
        if x0 >= x1 or y0 >= y1:
            continue
        # normalisation over the full truncated disk of this star
        v, u = np.mgrid[yi - rr:yi + rr + 1, xi - rr:xi + rr + 1].astype(np.float64)
        dx, dy = u - xs[i], v - ys[i]
        p = moffat_stamp(dx, dy, f, beta, e, t)
        p[dx * dx + dy * dy > rmax * rmax] = 0.0
        p *= fluxes[i] / p.sum()
        img[y0:y1, x0:x1] += p[y0 - (yi - rr):y1 - (yi - rr), x0 - (xi - rr):x1 - (xi - rr)]
    return img


def expose(rng: np.random.Generator, expected_e: np.ndarray, dark: np.ndarray,
           gain: float = 1.0, read_noise: float = READ_NOISE_E) -> np.ndarray:
    """Poisson + Gaussian read noise, to ADU, half-even rounding, uint16 clip."""
    counts = rng.poisson(np.maximum(expected_e, 0.0)).astype(np.float64)
    counts += rng.normal(0.0, read_noise, size=expected_e.shape)
    adu = np.rint(counts / gain + dark)
    return np.clip(adu, 0, SAT_ADU).astype(np.uint16)


@dataclasses.dataclass
class FramePair:
    """One synthetic science frame plus its reference stack and masters."""
    W: int
    H: int
    sci_raw: np.ndarray          # uint16 [H][W]
    ref_raw: list                # list of uint16 [H][W] (1 or 5 frames)
    dark: np.ndarray             # float32 [H][W] ADU
    flat: np.ndarray             # float32 [H][W]
    bpm: np.ndarray              # uint8 [H][W]
    sky: float
    gain: float
    read_noise: float
    star_x: np.ndarray
    star_y: np.ndarray
    star_f: np.ndarray
    trans_x: np.ndarray          # int transient positions
    trans_y: np.ndarray
    trans_f: np.ndarray
    fwhm_sci: object             # callable x -> FWHM of the science PSF
    fwhm_ref: object
    scale: float                 # science / reference flux ratio


def _masters(rng, W, H, realistic: bool):
    if not realistic:
        return (np.zeros((H, W), np.float32), np.ones((H, W), np.float32),
                np.zeros((H, W), np.uint8), np.zeros((H, W), bool))
    n = W * H
    dark = np.full(n, 100.0)
    hot = rng.random(n) < 5e-4
    dark[hot] += rng.uniform(50.0, 5000.0, hot.sum())
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    r2 = (xx - (W - 1) / 2.0) ** 2 + (yy - (H - 1) / 2.0) ** 2
    flat = (1.0 - 0.15 * r2 / r2.max()) * (1.0 + 0.01 * rng.standard_normal((H, W)))
    bpm = (rng.random(n) < 1e-4).astype(np.uint8)
    stuck_high = rng.random(n) < 0.5        # a bad pixel reads 65535 or 0
    return (dark.reshape(H, W).astype(np.float32), flat.astype(np.float32),
            bpm.reshape(H, W), stuck_high.reshape(H, W))


def make_pair(W: int = 1024, H: int = 1024, n_stars: int = 3000, seed: int = 1,
              fwhm_ref=2.0, fwhm_sci=2.6, varying_seeing: bool = False,
              n_ref: int = 1, realistic_masters: bool = False,
              sky: float = 800.0, scale: float = 1.05, n_transients: int = 20,
              cosmic_rate: float = 0.0, gain: float = 1.0) -> FramePair:
    """Draw one science frame and ``n_ref`` reference frames of the same scene.

    ``varying_seeing`` makes the science FWHM grow linearly from 1.5 to 4.0 px
    across x, with the reference at 2.0/2.6 of it, so the science image stays
    broader than the reference everywhere."""
    ss = np.random.SeedSequence(seed).spawn(N_STREAMS)
    rs = np.random.default_rng(ss[_S_STARS])
    xs = rs.uniform(0, W, n_stars)
    ys = rs.uniform(0, H, n_stars)
    fl = draw_fluxes(rs, n_stars)
    if varying_seeing:
        def fs(x):
            return 1.5 + 2.5 * np.asarray(x, np.float64) / max(W - 1, 1)

        def fr(x):
            return fs(x) * (2.0 / 2.6)
    else:
        def fs(x, v=float(fwhm_sci)):
            return np.full(np.shape(x), v)

        def fr(x, v=float(fwhm_ref)):
            return np.full(np.shape(x), v)
    dark, flat, bpm, stuck_high = _masters(np.random.default_rng(ss[_S_MASTERS]), W, H, realistic_masters)
    rt = np.random.default_rng(ss[_S_TRANS])
    margin = 32
    if n_transients > 0:
        tx = rt.integers(margin, W - margin, n_transients)
        ty = rt.integers(margin, H - margin, n_transients)
        tf = np.exp(rt.uniform(np.log(1e3), np.log(1e5), n_transients))
    else:
        tx = ty = np.zeros(0, np.int64)
        tf = np.zeros(0)
    ref_scene = render_scene(W, H, xs, ys, fl, fr)
    sci_scene = render_scene(W, H, np.concatenate([xs, tx.astype(np.float64)]),
                             np.concatenate([ys, ty.astype(np.float64)]),
                             np.concatenate([scale * fl, tf]), fs)
    flat64 = flat.astype(np.float64)
    dark64 = dark.astype(np.float64)
    bad = bpm != 0

    def frame(idx, scene, cosmics):
        rf = np.random.default_rng(ss[_S_FRAME0 + idx])
        e = flat64 * (sky + scene)
        if cosmics > 0:
            hit = np.flatnonzero(rf.random(e.size) < cosmics)
            e.reshape(-1)[hit] += rf.uniform(500.0, 2e4, hit.size)
        raw = expose(rf, e, dark64, gain)
        if bad.any():
            raw[bad & stuck_high] = SAT_ADU
            raw[bad & ~stuck_high] = 0
        return raw

    sci = frame(0, sci_scene, 0.0)
    refs = [frame(1 + i, ref_scene, cosmic_rate) for i in range(n_ref)]
    return FramePair(W, H, sci, refs, dark, flat, bpm, sky, gain, READ_NOISE_E,
                     xs, ys, fl, tx, ty, tf, fs, fr, scale)


def config1_pair(seed: int = 1, W: int = 1024, H: int = 1024, n_stars: int = 3000,
                 n_transients: int = 20) -> FramePair:
    """Plain CPU-sized pair: 1024^2, 3000 stars, FWHM 2.0 / 2.6, unit masters."""
    return make_pair(W, H, n_stars, seed, 2.0, 2.6, False, 1, False, 800.0, 1.05,
                     n_transients)


def config2_pair(seed: int = 2, W: int = IMX455_W, H: int = IMX455_H,
                 n_stars: int = 60000) -> FramePair:
    """Full IMX455 pair: ~60k stars, seeing 1.5-4.0 px across x, dark/flat/bpm
    masters and a 5-frame reference stack with cosmic rays in every frame."""
    return make_pair(W, H, n_stars, seed, None, None, True, 5, True, 800.0, 1.05, 20,
                     cosmic_rate=1e-5)


def draw_cutouts(seed: int, W: int, H: int, star_x, star_y, n: int,
                 lmin: int = 64, lmax: int = 512):
    """Cutout windows centred on catalogue stars drawn without replacement.

    Side L = floor(lmin * (lmax/lmin)^U), U uniform on [0, 1); the window
    origin is clamped so the window lies inside the frame."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(N_STREAMS)[_S_CUT])
    idx = rng.choice(len(star_x), size=min(n, len(star_x)), replace=False)
    u = rng.random(idx.size)
    L = np.floor(lmin * (lmax / lmin) ** u).astype(np.int64)
    L = np.minimum(L, min(W, H))
    cx = np.asarray(star_x)[idx]
    cy = np.asarray(star_y)[idx]
    x0 = np.clip(np.round(cx).astype(np.int64) - L // 2, 0, W - L)
    y0 = np.clip(np.round(cy).astype(np.int64) - L // 2, 0, H - L)
    return x0, y0, L


def random_stack(seed: int, n: int, H: int, W: int, level: float = 1000.0,
                 var_level: float = 1000.0):
    """Plain Gaussian frames for coadd tests: (cal, var, mask) lists."""
    rng = np.random.default_rng(seed)
    cal = [(level + math.sqrt(var_level) * rng.standard_normal((H, W))).astype(np.float32)
           for _ in range(n)]
    var = [np.full((H, W), var_level, np.float32) * rng.uniform(0.9, 1.1, (H, W)).astype(np.float32)
           for _ in range(n)]
    mask = [np.zeros((H, W), np.uint8) for _ in range(n)]
    return cal, var, mask
