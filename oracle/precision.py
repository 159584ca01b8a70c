"""Emulation of a BF16x3 normal-equation assembly (TEST INFRASTRUCTURE ONLY).

The split-precision scheme of Henry, Tang & Heinecke (2019, "Leveraging the
bfloat16 artificial intelligence datatype for higher-precision computations"):
each operand x is written x = hi + lo with hi = bf16(x) and lo = bf16(x - hi)
(round to nearest even on the bit pattern), and a product is approximated by
hi*hi' + hi*lo' + lo*hi' (the lo*lo' term is dropped).  Here it is applied to
the weighted design matrix X' = sqrt(w) X and right-hand side, with the
products and sums in FP64, to predict the error scale a BF16x3 assembly of the
normal equations incurs.
"""
from __future__ import annotations

import numpy as np

from . import core


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def split(x):
    x = np.asarray(x, np.float32)
    hi = bf16_round(x)
    lo = bf16_round(x - hi)
    return hi.astype(np.float64), lo.astype(np.float64)


def fit_kernel_bf16x3(ref, ref_var, ref_mask, sci, sci_var, sci_mask, spec):
    """GLOBAL fit whose normal equations are assembled from BF16x3 products."""
    B = core.basis(spec)
    H, W = np.shape(ref)
    C = core.convolve(ref, B)
    phi = core.fit_set(ref_mask, sci_mask, ref_var, sci_var, spec.half_width)
    xt, yt = core.norm_coords(W, H)
    ys, xs = np.nonzero(phi)
    X = core.design_rows(C, xt, yt, ys, xs, spec)
    sw = 1.0 / np.sqrt(np.asarray(sci_var, np.float64)[ys, xs] + np.asarray(ref_var, np.float64)[ys, xs])
    Xw = X * sw[:, None]
    Sw = np.asarray(sci, np.float64)[ys, xs] * sw
    hi, lo = split(Xw)
    shi, slo = split(Sw)
    A = hi.T @ hi + hi.T @ lo + lo.T @ hi
    b = hi.T @ shi + hi.T @ slo + lo.T @ shi
    co, st = core.solve(A, b, ys.size)
    return co[None], np.array([st]), np.array([ys.size])
