"""Seeded synthetic frames drawn on the GPU with torch (same recipe as synth).

For workloads of many full frames (20 cameras x 61 MPix) the numpy generator
is too slow; this one draws the same kinds of inputs on the device: uniform
star positions, power-law fluxes (dN/df ~ f^-1.75 over 1e2..1e6 e-), Moffat
beta = 3 stars truncated at 8 FWHM and normalised over the truncated disk,
sky, Poisson + 1.7 e- read noise, half-even rounding to 16-bit ADU, the
same seed giving the same frames bit for bit.  It holds none of the
reduction's arithmetic.  Streams come from
numpy SeedSequence(seed) -> torch.Generator seeds.
"""
from __future__ import annotations

import math

import numpy as np

from .synth import READ_NOISE_E, SAT_ADU, moffat_alpha


def _gen(seed, k, device):
    import torch
    s = np.random.SeedSequence([seed, k]).generate_state(1, np.uint64)[0]
    g = torch.Generator(device=device)
    g.manual_seed(int(s) & ((1 << 62) - 1))
    return g


def render(W, H, xs, ys, fl, fwhm, device, chunk=2048, ell=0.0, theta=0.0):
    """Sum of truncated unit-sum Moffat stars (float32 [H][W], electrons).
    ell > 0 stretches the profile along position angle theta with axis ratio
    1 - ell at constant area (r^2 = q x'^2 + y'^2 / q, q = 1 - ell)."""
    import torch
    img = torch.zeros(H * W, dtype=torch.float32, device=device)
    R = int(math.ceil(8.0 * fwhm))
    off = torch.arange(-R, R + 1, device=device, dtype=torch.float32)
    alpha2 = moffat_alpha(fwhm) ** 2
    for i in range(0, xs.numel(), chunk):
        x = xs[i:i + chunk]
        y = ys[i:i + chunk]
        f = fl[i:i + chunk]
        xi = torch.round(x).to(torch.int64)
        yi = torch.round(y).to(torch.int64)
        dx = (xi[:, None] + off[None, :].to(torch.int64)).to(torch.float32) - x[:, None]
        dy = (yi[:, None] + off[None, :].to(torch.int64)).to(torch.float32) - y[:, None]
        if ell > 0.0:
            q = 1.0 - ell
            c, sn = math.cos(theta), math.sin(theta)
            xp = c * dx[:, None, :] + sn * dy[:, :, None]
            yp = -sn * dx[:, None, :] + c * dy[:, :, None]
            r2 = q * xp ** 2 + yp ** 2 / q
        else:
            r2 = dy[:, :, None] ** 2 + dx[:, None, :] ** 2
        p = (1.0 + r2 / alpha2) ** -3.0
        p = torch.where(r2 <= (8.0 * fwhm) ** 2, p, torch.zeros_like(p))
        p = p * (f / p.sum(dim=(1, 2)))[:, None, None]
        X = xi[:, None, None] + off[None, None, :].to(torch.int64)
        Y = yi[:, None, None] + off[None, :, None].to(torch.int64)
        ok = (X >= 0) & (X < W) & (Y >= 0) & (Y < H)
        idx = (Y * W + X)[ok]
        _add_at(img, idx, p[ok])
    return img.view(H, W)


def _add_at(img, idx, vals):
    """img[idx] += vals with repeated indices summed in a fixed order, so that
    the same seed always gives the same image: a float index_add_ on the device
    sums colliding contributions with atomics, in whatever order they land."""
    import torch
    if img.numel() < (1 << 31):
        idx = idx.to(torch.int32)          # narrower keys sort faster
    order = torch.argsort(idx, stable=True)
    uniq, counts = torch.unique_consecutive(idx[order], return_counts=True)
    sums = torch.segment_reduce(vals[order], "sum", lengths=counts)
    img.index_add_(0, uniq, sums)


def make_pair(W, H, n_stars, seed, fwhm_sci, ratio=2.0 / 2.6, sky=800.0, scale=1.05,
              device="cuda", ell=0.0, theta=0.0, noise_free=False):
    """Science and reference raw uint16 frames (device) plus star positions.
    The science PSF may be elliptical (ell, theta).  With noise_free the
    expected electron images (scene + sky, float32) are returned as two more
    values."""
    import torch
    g = _gen(seed, 0, device)
    xs = torch.rand(n_stars, generator=g, device=device, dtype=torch.float64) * W
    ys = torch.rand(n_stars, generator=g, device=device, dtype=torch.float64) * H
    u = torch.rand(n_stars, generator=g, device=device, dtype=torch.float64)
    a, b = 1e6 ** -0.75, 1e2 ** -0.75
    fl = (a + u * (b - a)) ** (-4.0 / 3.0)
    xs32, ys32, fl32 = xs.float(), ys.float(), fl.float()
    ref_scene = render(W, H, xs32, ys32, fl32, fwhm_sci * ratio, device)
    sci_scene = render(W, H, xs32, ys32, scale * fl32, fwhm_sci, device, ell=ell, theta=theta)

    def expose(scene, k):
        gk = _gen(seed, k, device)
        e = scene + sky
        cnt = torch.poisson(e, generator=gk)
        cnt = cnt + torch.randn(e.shape, generator=gk, device=device) * READ_NOISE_E
        adu = torch.clamp(torch.round(cnt), 0, SAT_ADU).to(torch.int32)
        return adu.to(torch.int16 if False else torch.int32)

    sci = expose(sci_scene, 1)
    ref = expose(ref_scene, 2)

    def u16(t):
        # values are in 0..65535: keep the low 16 bits as uint16
        return (t & 0xFFFF).to(torch.int16).view(torch.uint16)

    out = (u16(sci), u16(ref), xs.cpu().numpy(), ys.cpu().numpy())
    if noise_free:
        out += (sci_scene + sky, ref_scene + sky)
    return out
