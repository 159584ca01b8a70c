"""Emulation of the BF16x3 normal-equation assembly (TEST INFRASTRUCTURE ONLY).

The split-precision scheme of Henry, Tang & Heinecke (2019, "Leveraging the
bfloat16 artificial intelligence datatype for higher-precision
computations"): an operand x is written x = hi + lo with hi = bf16(x) and
lo = bf16(x - hi), both rounded to nearest even on the bit pattern, and a
product is approximated by hi*hi' + hi*lo' + lo*hi' (lo*lo' is dropped).

What is emulated is the moment form of the least-squares fit (the normal
equations A = sum w X X^T, b = sum w X S of the Transient Alerts section's
direct subtraction, with X the basis convolutions times spatial monomials):
every entry of A is a moment

    G_ab[k][l] = sum_p w xt^a yt^b c_k c_l,      a + b <= 2 D,

of the vector c = (C_0 .. C_{nb-1}, 1) (basis convolutions, then the
background's constant), and every entry of b a moment
R_ab[k] = sum_p w xt^a yt^b c_k S with a + b <= D.  The emulated arithmetic:

* operands in FP32: c_k = fp32(C_k) with C_k the FP64 convolution, the weight
  w = fp32(1 / fp32(var_S + var_R)), xt^a by repeated FP32 products,
  and the second factor B = fp32(fp32(w xt^a) c_l);
* per image row, the pixels are taken in segments of 64 columns (starting at
  the first interior column of the region); in each segment and for each
  power a, c_k and B are split into bf16 hi/lo and the three products are
  accumulated in FP32 over two steps of 32 pixels (each step's sum of
  32 products formed exactly and rounded once into the FP32 accumulator, in
  the order hi.hi, hi.lo, lo.hi);
* the FP32 segment sums are multiplied by yt^b and added in FP64;
* the right-hand side is formed from the FP32 operands in FP64 (its own
  FP32 rounding sits far below the split error), and the system is solved in
  FP64 by the oracle's Jacobi-scaled Cholesky.

Only G[k][l] with k <= l is formed (A operand c_k, B operand of c_l); the
lower triangle is its mirror.  With split=False the same code forms the
moments without the split (FP64 products and sums), and with
fp32_operands=False it skips the FP32 rounding of the operands: both switches
off give the FP64 normal equations in moment form.
"""
from __future__ import annotations

import numpy as np

from . import core

SEG = 64          # pixels of one row segment (one FP32 accumulation)
STEP = 32         # pixels of one accumulation step


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    b = np.ascontiguousarray(x, np.float32).view(np.uint32)
    lsb = (b >> np.uint32(16)) & np.uint32(1)
    # finite inputs stay below 2^32 after the increment (|x| < 2^128)
    r = ((b + np.uint32(0x7FFF) + lsb) >> np.uint32(16)) << np.uint32(16)
    return r.view(np.float32)


def split(x):
    """(hi, lo) as float64 with hi = bf16(x), lo = bf16(x - hi), x taken in FP32."""
    x = np.asarray(x, np.float32)
    hi = bf16_round(x)
    lo = bf16_round(x - hi)
    return hi.astype(np.float64), lo.astype(np.float64)


def _f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def segment_moments(c, B, split_products=True):
    """FP32 segment sums of c_k B_l.

    c: [N][SEG][32] first operands, B: [N][SEG][32] second operands (already
    rounded as the caller wants them).  Returns [N][32][32] float64 holding the
    FP32 accumulator after the segment: for each 32-pixel step in turn, the
    exact step sums of hi.hi, hi.lo and lo.hi are each rounded into it
    (split_products), or the exact FP64 sum over the segment (otherwise)."""
    c = np.asarray(c, np.float64)
    B = np.asarray(B, np.float64)
    if not split_products:
        return np.matmul(c.transpose(0, 2, 1), B)
    ch, cl = split(c)
    bh, bl = split(B)
    acc = np.zeros((c.shape[0], c.shape[2], B.shape[2]), np.float32)
    for s0 in range(0, c.shape[1], STEP):
        sl = slice(s0, s0 + STEP)
        for A_, B_ in ((ch, bh), (ch, bl), (cl, bh)):
            part = np.matmul(A_[:, sl].transpose(0, 2, 1), B_[:, sl])
            acc = (acc.astype(np.float64) + part).astype(np.float32)
    return acc.astype(np.float64)


def moment_system(ref, ref_var, ref_mask, sci, sci_var, sci_mask, spec, split_products=True,
                  fp32_operands=True, C=None):
    """Normal equations per solve from the emulated moments.  C, if given, is
    the FP64 stack of basis convolutions of ref (core.convolve(ref, basis)).

    Returns (A [n_solves][n][n], b [n_solves][n], n_fit [n_solves])."""
    B = core.basis(spec)
    nb = B.shape[0]
    H, W = np.shape(ref)
    h = spec.half_width
    D, Dbg = spec.spatial_degree, spec.bg_degree
    NA = 2 * D + 1
    rd = _f32 if fp32_operands else (lambda x: np.asarray(x, np.float64))
    C = core.convolve(ref, B) if C is None else C             # [nb][H][W], NaN at the border
    phi = core.fit_set(ref_mask, sci_mask, ref_var, sci_var, h)
    tot = rd(rd(sci_var) + rd(ref_var))
    with np.errstate(all="ignore"):
        w = np.where(phi, rd(1.0 / np.where(phi, tot, 1.0)), 0.0)
    s = rd(sci)
    xt, yt = core.norm_coords(W, H)
    xtr = rd(xt)
    xpw = [np.ones(W)]
    for _ in range(1, NA):
        xpw.append(rd(xpw[-1] * xtr))
    mons = core.monomials(D)
    monb = core.monomials(Dbg)
    nP = len(mons)
    n = nb * nP + len(monb)
    if spec.mode == core.GLOBAL:
        regions = [(0, W, 0, H)]
    else:
        regions = core._solve_regions(spec, W, H)
    As = np.zeros((len(regions), n, n))
    bs = np.zeros((len(regions), n))
    nf = np.zeros(len(regions), np.int64)
    for t, (x0, x1, y0, y1) in enumerate(regions):
        ix0, ix1 = max(x0, h), min(x1, W - h)
        iy0, iy1 = max(y0, h), min(y1, H - h)
        if ix0 >= ix1 or iy0 >= iy1:
            continue
        nf[t] = int(phi[iy0:iy1, ix0:ix1].sum())
        nseg = (ix1 - ix0 + SEG - 1) // SEG
        xs = ix0 + np.arange(nseg * SEG)
        inx = xs < ix1
        xs = np.minimum(xs, ix1 - 1)
        G = np.zeros((NA, 2 * D + 1, 32, 32))                 # [a][b][k][l]
        R = np.zeros((D + 1, D + 1, 32))                      # [a][b][k]
        for ya in range(iy0, iy1, 64):                        # rows in chunks (memory)
            yb = min(ya + 64, iy1)
            ys = np.arange(ya, yb)
            cv = np.zeros((ys.size, xs.size, 32))
            cv[:, :, :nb] = rd(C[:, ys][:, :, xs]).transpose(1, 2, 0)
            cv[:, :, nb] = 1.0
            wv = np.where(inx[None, :], w[np.ix_(ys, xs)], 0.0)
            ypw = np.stack([yt[ys] ** b for b in range(2 * D + 1)], 1)     # FP64 yt^b
            cseg = cv.reshape(ys.size * nseg, SEG, 32)
            for a in range(NA):
                wx = rd(wv * xpw[a][xs][None, :])
                Bop = rd(wx[:, :, None] * cv)
                m = segment_moments(cseg, Bop.reshape(ys.size * nseg, SEG, 32), split_products)
                mrow = m.reshape(ys.size, nseg, 32, 32).sum(1)   # FP64 sum of the segments
                for b in range(2 * D + 1 - a):
                    G[a, b] += np.tensordot(ypw[:, b], mrow, axes=1)
            for a in range(D + 1):
                ws = rd(rd(wv * s[np.ix_(ys, xs)]) * xpw[a][xs][None, :])
                r = np.einsum("yx,yxk->yk", ws, cv)
                for b in range(D + 1 - a):
                    R[a, b] += ypw[:, b] @ r
        # unknown (k, m): basis k times P_m = xt^p yt^q; background m: component nb
        rows = [(k, p, q) for k in range(nb) for (p, q) in mons] + [(nb, p, q) for (p, q) in monb]

        def gram(a, b, k, l):
            return G[a, b, min(k, l), max(k, l)]

        for i, (k, p, q) in enumerate(rows):
            bs[t, i] = R[p, q, k]
            for j, (l, p2, q2) in enumerate(rows):
                As[t, i, j] = gram(p + p2, q + q2, k, l)
    return As, bs, nf


def fit_kernel_bf16x3(ref, ref_var, ref_mask, sci, sci_var, sci_mask, spec, split_products=True,
                      fp32_operands=True, C=None):
    """Kernel fit whose normal equations come from the emulated moments.
    Returns (coeffs [n_solves][n], status [n_solves], n_fit [n_solves])."""
    A, b, nf = moment_system(ref, ref_var, ref_mask, sci, sci_var, sci_mask, spec,
                             split_products, fp32_operands, C)
    co = np.zeros(b.shape)
    st = np.zeros(b.shape[0], np.int32)
    for s in range(b.shape[0]):
        co[s], st[s] = core.solve(A[s], b[s], nf[s])
    return co, st, nf
