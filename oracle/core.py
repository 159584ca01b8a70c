"""FP64 oracle: calibration, coadd, kernel basis, fit, subtraction, detection.

TEST INFRASTRUCTURE ONLY (see the package docstring): nothing on the product
path imports this module.

Conventions (the paper fixes none of them; each is a stated reading):

* images are [y][x], x fastest; pixel (x, y) has its centre at integer
  coordinates; units are ADU, and electrons when gain = 1;
* convolution is true convolution, (R (x) K)(x, y) = sum_{u,v=-h..h}
  K(u, v) R(x-u, y-v), stamps stored K[v+h][u+h];
* normalised coordinates xt = (2x - (W-1))/(W-1), yt likewise, in [-1, 1];
* spatial monomials P_m = xt^p yt^q ordered p = 0..D outer, q = 0..D-p inner;
* mask bits BAD 0x01, SAT 0x02, EDGE 0x04, NODATA 0x08, FOOT 0x10,
  DET 0x20, CAND 0x40.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

BAD, SAT, EDGE, NODATA, FOOT, DET, CAND = 0x01, 0x02, 0x04, 0x08, 0x10, 0x20, 0x40

GLOBAL, PER_TILE = 0, 1


# ---------------------------------------------------------------------------
# Calibration: dark subtraction, flat fielding, bad-pixel masking
# (Image Management section; calibration sets of the Compute Nodes section).
# ---------------------------------------------------------------------------
def calibrate(raw, dark, flat, bpm, gain=1.0, read_noise=1.7, sat_adu=65535):
    """cal = (raw - dark)/flat,  var = (max(raw - dark, 0)/g + RN^2/g^2)/flat^2.

    The dark master holds the bias.  The variance is the CCD noise equation
    (shot noise of the dark-subtracted signal plus read noise, Table 1's
    1.7 e-), carried through the flat; it is the per-pixel noise map the
    Compute Nodes section keeps next to each calibration set.

    mask: BAD where bpm != 0, flat <= 0, or flat/dark is not finite;
          SAT where raw >= sat_adu.  BAD pixels get cal = var = 0.
    """
    raw = np.asarray(raw).astype(np.float64)
    dark = np.asarray(dark).astype(np.float64)
    flat = np.asarray(flat).astype(np.float64)
    bpm = np.zeros(raw.shape, np.uint8) if bpm is None else np.asarray(bpm)
    bad = (bpm != 0) | ~np.isfinite(flat) | ~np.isfinite(dark) | ~(flat > 0)
    mask = np.where(bad, BAD, 0).astype(np.uint8)
    mask |= np.where(raw >= sat_adu, SAT, 0).astype(np.uint8)
    with np.errstate(all="ignore"):
        sig = raw - dark
        cal = sig / flat
        var = (np.maximum(sig, 0.0) / gain + read_noise ** 2 / gain ** 2) / (flat * flat)
    cal[bad] = 0.0
    var[bad] = 0.0
    return cal, var, mask


# ---------------------------------------------------------------------------
# Reference coadd: iterative kappa-sigma clip about the median, sigma taken
# from the noise model (Deep Coaddition / Transient Alerts sections).
# ---------------------------------------------------------------------------
def coadd(cals, vars_, masks, kappa=3.0, max_iter=5, return_margin=False):
    """Clipped mean of n registered calibrated frames, per pixel.

    Reading: a sigma estimated from the same five samples can never reject one
    at 3 sigma (Samuelson's inequality bounds |x_i - median| by 3 sample
    sigmas for n = 5), so the clip uses the noise model: sigma^2 = median of
    the per-frame variances of the surviving samples.

      S = frames whose mask has neither BAD nor SAT
      repeat up to max_iter times:
          stop if |S| <= 2
          c = median(x_S), s2 = median(v_S)   (even count: mean of middle two)
          Rej = {i in S : |x_i - c| > kappa * sqrt(s2)}
          stop if Rej is empty, or if fewer than 2 would survive
          S = S minus Rej
      ref = mean(x_S), ref_var = sum(v_S)/|S|^2, n_used = |S|
      ref_mask: NODATA where S starts empty (ref = ref_var = 0);
                SAT where any input frame is SAT.

    With return_margin, also returns per pixel the smallest relative distance
    | |x_i - c| - kappa sigma | / (kappa sigma) over the samples and passes
    the clip evaluated (inf where it never ran): where it is tiny, inputs
    that differ by rounding may be clipped differently.
    """
    x = np.stack([np.asarray(c, np.float64) for c in cals])
    v = np.stack([np.asarray(c, np.float64) for c in vars_])
    m = np.stack([np.asarray(c, np.uint8) for c in masks])
    S = (m & (BAD | SAT)) == 0
    active = np.ones(x.shape[1:], bool)
    margin = np.full(x.shape[1:], np.inf)
    with np.errstate(all="ignore"):
        for _ in range(max_iter):
            cnt = S.sum(0)
            active &= cnt > 2
            if not active.any():
                break
            c = np.nanmedian(np.where(S, x, np.nan), axis=0)
            s2 = np.nanmedian(np.where(S, v, np.nan), axis=0)
            ks = kappa * np.sqrt(s2)
            if return_margin:
                rel = np.abs(np.abs(x - c) - ks) / ks
                rel = np.where(S & active, rel, np.inf).min(0)
                margin = np.minimum(margin, np.where(np.isnan(rel), 0.0, rel))
            rej = S & (np.abs(x - c) > ks) & active
            nrej = rej.sum(0)
            active &= nrej > 0
            active &= (cnt - nrej) >= 2
            S = S & ~(rej & active)
        cnt = S.sum(0)
        ref = np.where(cnt > 0, np.where(S, x, 0.0).sum(0) / np.maximum(cnt, 1), 0.0)
        ref_var = np.where(cnt > 0, np.where(S, v, 0.0).sum(0) / np.maximum(cnt, 1) ** 2, 0.0)
    ref_mask = np.where(cnt == 0, NODATA, 0).astype(np.uint8)
    ref_mask |= np.where(((m & SAT) != 0).any(0), SAT, 0).astype(np.uint8)
    if return_margin:
        return ref, ref_var, ref_mask, cnt.astype(np.uint8), margin
    return ref, ref_var, ref_mask, cnt.astype(np.uint8)


# ---------------------------------------------------------------------------
# Kernel basis: Gaussians times polynomials (Alard & Lupton 1998), with the
# flux-normalised combination of Alard (2000).
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class KernelSpec:
    sigmas: tuple = (0.7, 1.5, 3.0)
    degrees: tuple = (4, 3, 2)
    half_width: int = 7
    spatial_degree: int = 0
    bg_degree: int = 0
    tiles_x: int = 1
    tiles_y: int = 1
    mode: int = GLOBAL


def basis_meta(spec):
    """(g, i, j) of each basis function: g outer, then i, then j."""
    out = []
    for g, d in enumerate(spec.degrees):
        for i in range(d + 1):
            for j in range(d - i + 1):
                out.append((g, i, j))
    return out


def basis(spec):
    """Basis stamps B[k][v+h][u+h], float64.

    B_k(u, v) = exp(-(u^2+v^2)/(2 sigma_g^2)) u^i v^j on the integer grid.
    Normalisation (spans unchanged):
      1. B_0 scaled to unit sum;
      2. every k >= 1 with i and j both even becomes B_k - (sum B_k) B_0;
      3. every k >= 1 scaled to unit L2 norm.
    Afterwards every k >= 1 sums to zero, so the kernel sum equals the
    coefficient of B_0 (the photometric scale factor).
    """
    h = spec.half_width
    v, u = np.mgrid[-h:h + 1, -h:h + 1].astype(np.float64)
    meta = basis_meta(spec)
    B = np.empty((len(meta), 2 * h + 1, 2 * h + 1))
    for k, (g, i, j) in enumerate(meta):
        s = spec.sigmas[g]
        B[k] = np.exp(-(u * u + v * v) / (2.0 * s * s)) * u ** i * v ** j
    B[0] /= B[0].sum()
    for k, (g, i, j) in enumerate(meta):
        if k == 0:
            continue
        if i % 2 == 0 and j % 2 == 0:
            B[k] = B[k] - B[k].sum() * B[0]
        B[k] /= math.sqrt((B[k] * B[k]).sum())
    return B


def convolve(img, K):
    """Direct 2-D true convolution, (img (x) K)(x, y) = sum K(u,v) img(x-u, y-v).

    K may be one stamp [2h+1][2h+1] or a stack [n][2h+1][2h+1].  The result
    has the image's shape; pixels within h of the border (where the sum would
    leave the image) are NaN.  Evaluated in row chunks as a tensordot of the
    sliding windows with the flipped stamps, which is the sum written out.
    """
    img = np.asarray(img, np.float64)
    K = np.asarray(K, np.float64)
    single = K.ndim == 2
    if single:
        K = K[None]
    n, kh, kw = K.shape
    h = kh // 2
    H, W = img.shape
    out = np.full((n, H, W), np.nan)
    if H < kh or W < kw:
        return out[0] if single else out
    Kf = K[:, ::-1, ::-1].reshape(n, -1)              # window tap (a, b) pairs with K[2h-a][2h-b]
    Wo = W - 2 * h
    step = max(1, (1 << 14) // Wo)
    for y0 in range(0, H - 2 * h, step):
        y1 = min(y0 + step, H - 2 * h)
        cols = np.empty((kh * kw, (y1 - y0) * Wo))   # cols[(a, b)] = img[y + a - h, x + b - h]
        for a in range(kh):
            for b in range(kw):
                cols[a * kw + b] = img[y0 + a:y1 + a, b:b + Wo].ravel()
        out[:, y0 + h:y1 + h, h:W - h] = (Kf @ cols).reshape(n, y1 - y0, Wo)
    return out[0] if single else out


# ---------------------------------------------------------------------------
# Spatial polynomial, tiles, fit set, design matrix, normal equations.
# ---------------------------------------------------------------------------
def monomials(D):
    """(p, q) exponents of P_m = xt^p yt^q, p = 0..D outer, q = 0..D-p inner."""
    return [(p, q) for p in range(D + 1) for q in range(D - p + 1)]


def norm_coords(W, H):
    """xt[x], yt[y] in [-1, 1]; a 1-pixel axis maps to 0."""
    xt = (2.0 * np.arange(W) - (W - 1)) / (W - 1) if W > 1 else np.zeros(1)
    yt = (2.0 * np.arange(H) - (H - 1)) / (H - 1) if H > 1 else np.zeros(1)
    return xt, yt


def tile_bounds(n_pix, n_tiles):
    """Tile i spans [floor(i n/T), floor((i+1) n/T))."""
    return [(i * n_pix // n_tiles, (i + 1) * n_pix // n_tiles) for i in range(n_tiles)]


def n_unknowns(spec):
    nb = len(basis_meta(spec))
    nP = len(monomials(spec.spatial_degree))
    nPb = len(monomials(spec.bg_degree))
    return nb * nP + nPb


def footprint_clean(ref_mask, h):
    """True where ref_mask == 0 over the whole (2h+1)^2 footprint (interior only)."""
    H, W = ref_mask.shape
    ok = np.zeros((H, W), bool)
    if H < 2 * h + 1 or W < 2 * h + 1:
        return ok
    win = sliding_window_view(ref_mask != 0, (2 * h + 1, 2 * h + 1))
    ok[h:H - h, h:W - h] = ~win.any(axis=(2, 3))
    return ok


def fit_set(ref_mask, sci_mask, ref_var, sci_var, h):
    """Pixels that enter the fit: interior (h <= x <= W-1-h, same in y),
    sci_mask == 0, ref_mask == 0 over the footprint, var_S + var_R > 0."""
    ok = footprint_clean(np.asarray(ref_mask), h)
    ok &= np.asarray(sci_mask) == 0
    ok &= (np.asarray(sci_var, np.float64) + np.asarray(ref_var, np.float64)) > 0
    return ok


def _solve_regions(spec, W, H):
    """List of (x0, x1, y0, y1) per solve; GLOBAL is one region of all tiles."""
    tx = tile_bounds(W, spec.tiles_x)
    ty = tile_bounds(H, spec.tiles_y)
    return [(x0, x1, y0, y1) for (y0, y1) in ty for (x0, x1) in tx]


def design_rows(C, xt, yt, ys, xs, spec):
    """Rows X_p for the pixels (ys, xs): [P_m C_k] at index k*nP + m, then [P_m]
    for the background block (m < nP(D_bg)).  C is the [nb][H][W] stack of
    basis convolutions."""
    mons = monomials(spec.spatial_degree)
    monb = monomials(spec.bg_degree)
    nb = C.shape[0]
    nP = len(mons)
    X = np.empty((ys.size, nb * nP + len(monb)))
    P = np.stack([xt[xs] ** p * yt[ys] ** q for (p, q) in mons], 1)
    Pb = np.stack([xt[xs] ** p * yt[ys] ** q for (p, q) in monb], 1)
    Cp = C[:, ys, xs].T                              # [npix][nb]
    for k in range(nb):
        X[:, k * nP:(k + 1) * nP] = Cp[:, k:k + 1] * P
    X[:, nb * nP:] = Pb
    return X


def normal_equations(ref, ref_var, ref_mask, sci, sci_var, sci_mask, spec, B=None, C=None,
                     coords=None):
    """Per tile t: A_t = sum w X X^T, b_t = sum w X S over the fit set in t,
    with w = 1/(var_S + var_R).  Returns (A [T][n][n], b [T][n], n_fit [T])
    for the tiles in raster order.  C, if given, is convolve(ref, B); coords,
    if given, are the (xt, yt) arrays of these columns and rows when the
    images are a window of a larger frame (its normalised coordinates)."""
    B = basis(spec) if B is None else B
    H, W = np.shape(ref)
    h = spec.half_width
    C = convolve(ref, B) if C is None else C
    phi = fit_set(ref_mask, sci_mask, ref_var, sci_var, h)
    xt, yt = norm_coords(W, H) if coords is None else coords
    sci = np.asarray(sci, np.float64)
    wts = 1.0 / (np.asarray(sci_var, np.float64) + np.asarray(ref_var, np.float64) + (~phi))
    n = n_unknowns(spec)
    tiles = [(x0, x1, y0, y1) for (y0, y1) in tile_bounds(H, spec.tiles_y)
             for (x0, x1) in tile_bounds(W, spec.tiles_x)]
    A = np.zeros((len(tiles), n, n))
    b = np.zeros((len(tiles), n))
    nf = np.zeros(len(tiles), np.int64)
    for t, (x0, x1, y0, y1) in enumerate(tiles):
        ys, xs = np.nonzero(phi[y0:y1, x0:x1])
        ys = ys + y0
        xs = xs + x0
        nf[t] = ys.size
        if ys.size == 0:
            continue
        X = design_rows(C, xt, yt, ys, xs, spec)
        wv = wts[ys, xs]
        A[t] = X.T @ (wv[:, None] * X)
        b[t] = X.T @ (wv * sci[ys, xs])
    return A, b, nf


def cholesky(A):
    """Plain column Cholesky A = L L^T.  Returns (L, pivots) where pivots[j] is
    the diagonal of the Schur complement before its square root; L is only
    valid when every pivot is positive."""
    A = np.array(A, np.float64)
    n = A.shape[0]
    L = np.zeros_like(A)
    piv = np.zeros(n)
    for j in range(n):
        s = A[j, j] - L[j, :j] @ L[j, :j]
        piv[j] = s
        if not s > 0:
            return L, piv
        L[j, j] = math.sqrt(s)
        L[j + 1:, j] = (A[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L, piv


STATUS_OK, STATUS_SINGULAR, STATUS_TOOFEW = 0, -20, -21


def solve(A, b, n_fit):
    """Jacobi-scaled Cholesky solve of A a = b.

    d = diag(A)^-1/2, A' = d A d, b' = d b.  TOOFEW if n_fit < n; SINGULAR if a
    diagonal is not positive or a pivot is <= n 2^-52 max diag(A').  Failed
    solves return NaN coefficients."""
    A = np.asarray(A, np.float64)
    b = np.asarray(b, np.float64)
    n = A.shape[0]
    if n_fit < n:
        return np.full(n, np.nan), STATUS_TOOFEW
    dg = np.diag(A)
    if not np.all(dg > 0):
        return np.full(n, np.nan), STATUS_SINGULAR
    d = 1.0 / np.sqrt(dg)
    As = A * d[:, None] * d[None, :]
    bs = b * d
    L, piv = cholesky(As)
    if np.any(piv <= n * 2.0 ** -52 * np.max(np.diag(As))):
        return np.full(n, np.nan), STATUS_SINGULAR
    z = np.zeros(n)
    for i in range(n):
        z[i] = (bs[i] - L[i, :i] @ z[:i]) / L[i, i]
    y = np.zeros(n)
    for i in range(n - 1, -1, -1):
        y[i] = (z[i] - L[i + 1:, i] @ y[i + 1:]) / L[i, i]
    return d * y, STATUS_OK


def fit_kernel(ref, ref_var, ref_mask, sci, sci_var, sci_mask, spec, B=None, C=None):
    """Least-squares kernel fit.  GLOBAL: the tile sums are added in raster
    order and solved once.  PER_TILE: one solve per tile.  C, if given, is the
    stack of basis convolutions of ref.
    Returns (coeffs [n_solves][n], status [n_solves], n_fit [n_solves])."""
    A, b, nf = normal_equations(ref, ref_var, ref_mask, sci, sci_var, sci_mask, spec, B, C)
    if spec.mode == GLOBAL:
        As = np.zeros(A.shape[1:])
        bs = np.zeros(b.shape[1:])
        for t in range(A.shape[0]):
            As += A[t]
            bs += b[t]
        A, b, nf = As[None], bs[None], np.array([nf.sum()])
    co = np.zeros(b.shape)
    st = np.zeros(b.shape[0], np.int32)
    for s in range(b.shape[0]):
        co[s], st[s] = solve(A[s], b[s], nf[s])
    return co, st, nf


def chi2(ref, ref_var, ref_mask, sci, sci_var, sci_mask, spec, coeffs, B=None):
    """chi^2 = sum over the fit set of w (S - X a)^2, as a second pass over the
    residuals.  One value per solve; dof = n_fit - n."""
    B = basis(spec) if B is None else B
    H, W = np.shape(ref)
    C = convolve(ref, B)
    phi = fit_set(ref_mask, sci_mask, ref_var, sci_var, spec.half_width)
    xt, yt = norm_coords(W, H)
    sci = np.asarray(sci, np.float64)
    wts = 1.0 / (np.asarray(sci_var, np.float64) + np.asarray(ref_var, np.float64) + (~phi))
    tiles = _solve_regions(spec, W, H)
    out = np.zeros(len(coeffs))
    for t, (x0, x1, y0, y1) in enumerate(tiles):
        s = 0 if spec.mode == GLOBAL else t
        ys, xs = np.nonzero(phi[y0:y1, x0:x1])
        ys = ys + y0
        xs = xs + x0
        if ys.size == 0:
            continue
        X = design_rows(C, xt, yt, ys, xs, spec)
        r = sci[ys, xs] - X @ coeffs[s]
        out[s] += np.sum(wts[ys, xs] * r * r)
    return out


# ---------------------------------------------------------------------------
# Expansion, PSF-matched convolution and subtraction.
# ---------------------------------------------------------------------------
def expand_kernel(coeffs, spec, B=None):
    """K_m = sum_k a_{k nP + m} B_k and bg_m = a_{nb nP + m}.
    Returns (stamps [n_solves][nP][2h+1][2h+1], bg [n_solves][nPb])."""
    B = basis(spec) if B is None else B
    coeffs = np.atleast_2d(np.asarray(coeffs, np.float64))
    nb = B.shape[0]
    nP = len(monomials(spec.spatial_degree))
    st = np.einsum("skm,kvu->smvu", coeffs[:, :nb * nP].reshape(-1, nb, nP), B)
    return st, coeffs[:, nb * nP:]


def subtract(stamps, bg, ref, ref_var, ref_mask, sci, sci_var, sci_mask, spec, coords=None):
    """Per output pixel p (kernel evaluated at the output pixel):

      K_p = sum_m P_m(p) K_m   (K_m of the solve that owns p)
      M   = sum_{u,v} K_p(u,v) R(x-u, y-v) + sum_m bg_m P_m(p)
      D   = S - M
      V   = var_S + sum_{u,v} K_p(u,v)^2 var_R(x-u, y-v)

    diff_mask = sci_mask bits, plus EDGE within h of the border, plus FOOT where
    any ref_mask bit is set in the footprint; D = V = 0 wherever diff_mask != 0.
    chi2[s] = sum over the fit set of solve s of D^2/(var_S + var_R).
    coords: as for normal_equations (a window of a larger frame).
    Returns (D, V, diff_mask, chi2 [n_solves], n_fit [n_solves])."""
    stamps = np.asarray(stamps, np.float64)
    bg = np.atleast_2d(np.asarray(bg, np.float64))
    if stamps.ndim == 3:
        stamps = stamps[None]
    ref = np.asarray(ref, np.float64)
    rv = np.asarray(ref_var, np.float64)
    sci = np.asarray(sci, np.float64)
    sv = np.asarray(sci_var, np.float64)
    H, W = ref.shape
    h = spec.half_width
    kw = 2 * h + 1
    mons = monomials(spec.spatial_degree)
    monb = monomials(spec.bg_degree)
    xt, yt = norm_coords(W, H) if coords is None else coords
    Dimg = np.zeros((H, W))
    Vimg = np.zeros((H, W))
    dmask = np.asarray(sci_mask, np.uint8).copy()
    edge = np.ones((H, W), bool)
    edge[h:H - h, h:W - h] = False
    dmask |= np.where(edge, EDGE, 0).astype(np.uint8)
    clean = footprint_clean(np.asarray(ref_mask), h)
    dmask |= np.where(~edge & ~clean, FOOT, 0).astype(np.uint8)
    regions = _solve_regions(spec, W, H)
    owner = np.zeros((H, W), np.int64)
    if spec.mode == PER_TILE:
        for t, (x0, x1, y0, y1) in enumerate(regions):
            owner[y0:y1, x0:x1] = t
    if H >= kw and W >= kw:
        wr = sliding_window_view(ref, (kw, kw))
        wv = sliding_window_view(rv, (kw, kw))
        for y in range(h, H - h):
            xs = np.arange(h, W - h)
            P = np.stack([xt[xs] ** p * yt[y] ** q for (p, q) in mons], 1)     # [nx][nP]
            Pb = np.stack([xt[xs] ** p * yt[y] ** q for (p, q) in monb], 1)
            own = owner[y, xs]
            M = np.empty(xs.size)
            Vr = np.empty(xs.size)
            cut = np.flatnonzero(np.diff(own)) + 1
            for a, b in zip(np.r_[0, cut], np.r_[cut, xs.size]):   # runs of one solve
                s = own[a]
                Kp = np.einsum("xm,mvu->xvu", P[a:b], stamps[s])   # K_p at each pixel
                Kf = Kp[:, ::-1, ::-1]                    # window tap (a, b) <-> K[2h-a][2h-b]
                M[a:b] = np.einsum("xab,xab->x", wr[y - h, a:b], Kf) + Pb[a:b] @ bg[s]
                Vr[a:b] = np.einsum("xab,xab->x", wv[y - h, a:b], Kf * Kf)
            Dimg[y, xs] = sci[y, xs] - M
            Vimg[y, xs] = sv[y, xs] + Vr
    bad = dmask != 0
    Dimg[bad] = 0.0
    Vimg[bad] = 0.0
    phi = fit_set(ref_mask, sci_mask, ref_var, sci_var, h)
    ns = len(stamps)
    c2 = np.zeros(ns)
    nf = np.zeros(ns, np.int64)
    with np.errstate(all="ignore"):
        wts = np.where(phi, 1.0 / (sv + rv), 0.0)
    for s in range(ns):
        sel = phi & (owner == s)
        c2[s] = np.sum(wts[sel] * Dimg[sel] ** 2)
        nf[s] = sel.sum()
    return Dimg, Vimg, dmask, c2, nf


def subtract_at(stamps, bg, ref, ref_var, ref_mask, sci, sci_var, sci_mask, spec, ys, xs):
    """The definitions of `subtract` evaluated at the pixels (ys, xs) only, in
    the frame's own coordinates, for frames too large to difference whole.
    Returns (D, V, diff_mask) at those pixels."""
    stamps = np.asarray(stamps, np.float64)
    bg = np.atleast_2d(np.asarray(bg, np.float64))
    if stamps.ndim == 3:
        stamps = stamps[None]
    ys = np.asarray(ys, np.int64)
    xs = np.asarray(xs, np.int64)
    H, W = np.shape(ref)
    h = spec.half_width
    mons = monomials(spec.spatial_degree)
    monb = monomials(spec.bg_degree)
    xt, yt = norm_coords(W, H)
    rm = np.asarray(ref_mask)
    ref = np.asarray(ref)
    ref_var = np.asarray(ref_var)
    dmask = np.asarray(sci_mask, np.uint8)[ys, xs].copy()
    edge = (xs < h) | (xs > W - 1 - h) | (ys < h) | (ys > H - 1 - h)
    dmask |= np.where(edge, EDGE, 0).astype(np.uint8)
    owner = np.zeros(ys.size, np.int64)
    if spec.mode == PER_TILE:
        for t, (x0, x1, y0, y1) in enumerate(_solve_regions(spec, W, H)):
            owner[(xs >= x0) & (xs < x1) & (ys >= y0) & (ys < y1)] = t
    D = np.zeros(ys.size)
    V = np.zeros(ys.size)
    off = np.arange(-h, h + 1)
    for i in np.flatnonzero(~edge):
        y, x = ys[i], xs[i]
        # win[a][b] = image(x + b - h, y + a - h), which K(u, v) meets at u = h - b, v = h - a
        if (rm[y - h:y + h + 1, x - h:x + h + 1] != 0).any():
            dmask[i] |= FOOT
        if dmask[i] != 0:
            continue
        s = owner[i]
        P = np.array([xt[x] ** p * yt[y] ** q for (p, q) in mons])
        Pb = np.array([xt[x] ** p * yt[y] ** q for (p, q) in monb])
        Kp = np.tensordot(P, stamps[s], axes=1)       # K_p[v+h][u+h]
        Kf = Kp[::-1, ::-1]
        wr = ref[np.ix_(y + off, x + off)].astype(np.float64)
        wv = ref_var[np.ix_(y + off, x + off)].astype(np.float64)
        D[i] = float(sci[y, x]) - ((wr * Kf).sum() + Pb @ bg[s])
        V[i] = float(sci_var[y, x]) + (wv * Kf * Kf).sum()
    return D, V, dmask


# ---------------------------------------------------------------------------
# Detection: noise-normalised difference, threshold, local maxima, PSF flux.
# ---------------------------------------------------------------------------
CAND_DTYPE = np.dtype([("x", np.int32), ("y", np.int32), ("snr", np.float64),
                       ("flux", np.float64), ("flux_err", np.float64)])


def detect(D, V, diff_mask, threshold, psf):
    """SNR = D/sqrt(V) where diff_mask == 0 and V > 0, else 0.
    DET where SNR >= threshold.  CAND where DET holds and SNR is strictly above
    every 8-neighbour earlier in raster order and >= every later one
    (out-of-image neighbours count as -inf), so a plateau keeps its
    raster-first pixel.  Per candidate, with the unit-sum PSF P of half-width
    r over unmasked in-image pixels of the window:
      Q = sum P^2/V,  flux = (sum P D/V)/Q,  flux_err = Q^-1/2.
    Candidates are sorted by y*W + x.  Returns (snr, det_mask, cands)."""
    D = np.asarray(D, np.float64)
    V = np.asarray(V, np.float64)
    dm = np.asarray(diff_mask)
    H, W = D.shape
    good = (dm == 0) & (V > 0)
    snr = np.zeros((H, W))
    with np.errstate(all="ignore"):
        snr[good] = D[good] / np.sqrt(V[good])
    det = snr >= threshold
    pad = np.full((H + 2, W + 2), -np.inf)
    pad[1:-1, 1:-1] = snr
    cand = det.copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            nb = pad[1 + dy:H + 1 + dy, 1 + dx:W + 1 + dx]
            earlier = dy < 0 or (dy == 0 and dx < 0)
            cand &= (snr > nb) if earlier else (snr >= nb)
    det_mask = np.where(det, DET, 0).astype(np.uint8) | np.where(cand, CAND, 0).astype(np.uint8)
    psf = np.asarray(psf, np.float64)
    r = psf.shape[0] // 2
    ys, xs = np.nonzero(cand)                         # row-major: raster order
    out = np.zeros(ys.size, CAND_DTYPE)
    for i, (y, x) in enumerate(zip(ys, xs)):
        q = f = 0.0
        for v in range(-r, r + 1):
            yy = y + v
            if yy < 0 or yy >= H:
                continue
            for u in range(-r, r + 1):
                xx = x + u
                if xx < 0 or xx >= W or not good[yy, xx]:
                    continue
                p = psf[v + r, u + r]
                q += p * p / V[yy, xx]
                f += p * D[yy, xx] / V[yy, xx]
        out[i] = (x, y, snr[y, x], f / q if q > 0 else np.nan, q ** -0.5 if q > 0 else np.nan)
    return snr, det_mask, out
