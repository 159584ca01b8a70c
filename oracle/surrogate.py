"""FP64 oracle of the learned kernel surrogate (TEST INFRASTRUCTURE ONLY).

A learned surrogate of the kernel fit: a small CNN that maps a
stack of paired star stamps of one sub-tile to the kernel coefficients, with
the plain least-squares fit as the fallback.  Written here from its
definition, in numpy float64:

* stamp selection - up to S positive reference local maxima per tile
  (strictly above earlier 8-neighbours in raster order, >= later ones),
  brightest first with raster order breaking ties, whose (2r+1)^2 stamp
  lies inside the frame and is unmasked in both frames, and whose peak is
  at least snr_min noise sigmas above the reference stamp's border median
  (every decision in FP64).  Each stamp has its border median subtracted; both stamps are
  divided by the background-subtracted reference stamp sum and scaled by a
  fixed 100;
* network - four 3x3 'same' convolutions (zero padding, cross-correlation)
  2 -> C -> C -> C -> C channels with bias and ReLU, a spatial mean, a mean
  over the valid stamps, and a linear head to the nb kernel coefficients;
* loss - mean squared error over the coefficients and the batch;
* Adam - beta = (0.9, 0.999), eps = 1e-8, bias-corrected.

The background coefficient is not predicted: normalised stamps carry no sky
level, so given a kernel K the background is the one-parameter weighted
least-squares value bg = sum w (S - K (x) R) / sum w over the fit set.
"""
from __future__ import annotations

import numpy as np

from . import core


# ------------------------------------------------------------------ stamps
def select_stamps(ref, ref_var, ref_mask, sci_mask, tiles_x, tiles_y, r=15, S=64,
                  snr_min=10.0, tie_tol=None):
    """Per tile (raster order of tiles) a list of up to S (y, x) stamp centres.

    Candidates are positive reference local maxima (strictly above the
    8-neighbours earlier in raster order, >= the later ones) whose
    (2r+1)^2 stamp lies inside the frame and whose peak stands snr_min noise
    sigmas above the tile's sky, the median of its unmasked reference pixels
    (no candidates when all are masked), ranked brightest first with raster
    order breaking ties.  Walking down the ranking a candidate is kept when
    its stamp is unmasked in both frames and (peak - border median of its
    reference stamp) / sqrt(var at the peak) >= snr_min; the walk stops at S.
    Every quantity is taken in FP64 (medians average the middle pair).

    With tie_tol set, also returns per tile the number of candidates whose
    sky or border test quantity lies within tie_tol * snr_min of snr_min:
    there an implementation that rounds differently may decide the other
    way (and every later stamp of the tile may shift)."""
    ref = np.asarray(ref, np.float64)
    var = np.asarray(ref_var, np.float64)
    H, W = ref.shape
    pad = np.full((H + 2, W + 2), -np.inf)
    pad[1:-1, 1:-1] = ref
    lm = ref > 0
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            nb = pad[1 + dy:H + 1 + dy, 1 + dx:W + 1 + dx]
            earlier = dy < 0 or (dy == 0 and dx < 0)
            lm &= (ref > nb) if earlier else (ref >= nb)
    bad = (np.asarray(ref_mask) != 0) | (np.asarray(sci_mask) != 0)
    out = []
    near = []
    for (y0, y1) in core.tile_bounds(H, tiles_y):
        for (x0, x1) in core.tile_bounds(W, tiles_x):
            un = ref[y0:y1, x0:x1][np.asarray(ref_mask)[y0:y1, x0:x1] == 0]
            if un.size == 0:
                out.append([])
                near.append(0)
                continue
            sky = np.median(un)
            ys, xs = np.nonzero(lm[y0:y1, x0:x1])
            ys, xs = ys + y0, xs + x0
            inside = (ys >= r) & (xs >= r) & (ys < H - r) & (xs < W - r)
            ys, xs = ys[inside], xs[inside]
            nt = 0
            with np.errstate(all="ignore"):
                vv = var[ys, xs]
                q = np.where(vv > 0, (ref[ys, xs] - sky) / np.sqrt(vv), -np.inf)
            above = q >= snr_min
            if tie_tol is not None:
                nt += int((np.abs(q - snr_min) <= tie_tol * snr_min).sum())
            cand = sorted(zip(ys[above], xs[above]), key=lambda p: (-ref[p[0], p[1]],
                                                                     p[0] * W + p[1]))
            keep = []
            for y, x in cand:
                if len(keep) == S:
                    break
                if bad[y - r:y + r + 1, x - r:x + r + 1].any():
                    continue
                m = border_median(ref[y - r:y + r + 1, x - r:x + r + 1])
                v = var[y, x]
                if not v > 0:
                    continue
                qb = (ref[y, x] - m) / np.sqrt(v)
                if tie_tol is not None and abs(qb - snr_min) <= tie_tol * snr_min:
                    nt += 1
                if qb >= snr_min:
                    keep.append((y, x))
            out.append(keep)
            near.append(nt)
    return (out, near) if tie_tol is not None else out


def border_median(st):
    b = np.concatenate([st[0, :], st[-1, :], st[1:-1, 0], st[1:-1, -1]])
    return np.median(b)


STAMP_SCALE = 100.0


def make_stamps(ref, sci, centres, r=15, S=64, scale=STAMP_SCALE):
    """Input tensor [T][S][2][2r+1][2r+1] and validity [T][S] for the centres.

    Both stamps lose their border medians and are divided by the reference
    stamp's remaining sum, then multiplied by a fixed scale (100) that puts
    the network's inputs near unit size (a 31x31 stamp of unit sum has values
    of order 1e-3, below what BF16 activations resolve next to O(0.1) biases)."""
    ref = np.asarray(ref, np.float64)
    sci = np.asarray(sci, np.float64)
    T = len(centres)
    n = 2 * r + 1
    X = np.zeros((T, S, 2, n, n))
    valid = np.zeros((T, S))
    for t, cs in enumerate(centres):
        for s, (y, x) in enumerate(cs):
            rs = ref[y - r:y + r + 1, x - r:x + r + 1]
            ss = sci[y - r:y + r + 1, x - r:x + r + 1]
            rs = rs - border_median(rs)
            ss = ss - border_median(ss)
            tot = rs.sum()
            if not tot > 0:
                continue
            X[t, s, 0] = scale * rs / tot
            X[t, s, 1] = scale * ss / tot
            valid[t, s] = 1.0
    return X, valid


# ------------------------------------------------------------------ network
def init_params(rng, C=32, cin=2, nout=31):
    """He-normal convolution weights, zero biases, a small head."""
    p = {}
    ch = [cin, C, C, C, C]
    for l in range(4):
        fan = ch[l] * 9
        p[f"w{l}"] = rng.standard_normal((ch[l + 1], ch[l], 3, 3)) * np.sqrt(2.0 / fan)
        p[f"b{l}"] = np.zeros(ch[l + 1])
    p["hw"] = rng.standard_normal((nout, C)) * np.sqrt(1.0 / C)
    p["hb"] = np.zeros(nout)
    return p


def conv3x3(a, w, b):
    """'same' cross-correlation with zero padding: a [N][Cin][H][W], w [Co][Cin][3][3]."""
    N, Ci, H, W = a.shape
    ap = np.zeros((N, Ci, H + 2, W + 2))
    ap[:, :, 1:-1, 1:-1] = a
    out = np.zeros((N, w.shape[0], H, W)) + b[None, :, None, None]
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("nchw,oc->nohw", ap[:, :, dy:dy + H, dx:dx + W], w[:, :, dy, dx])
    return out


def forward(p, X, valid):
    """Returns (out [T][nout], cache).  X [T][S][2][n][n], valid [T][S]."""
    T, S = valid.shape
    a = X.reshape(T * S, *X.shape[2:])
    cache = {"in": a}
    for l in range(4):
        z = conv3x3(a, p[f"w{l}"], p[f"b{l}"])
        a = np.maximum(z, 0.0)
        cache[f"z{l}"] = z
        cache[f"a{l}"] = a
    pool = a.mean(axis=(2, 3)).reshape(T, S, -1)             # [T][S][C]
    nv = np.maximum(valid.sum(1), 1.0)
    q = (pool * valid[:, :, None]).sum(1) / nv[:, None]      # [T][C]
    out = q @ p["hw"].T + p["hb"][None, :]
    cache.update(pool=pool, q=q, nv=nv, valid=valid)
    return out, cache


def loss(out, target):
    return float(np.mean((out - target) ** 2))


def backward(p, cache, out, target):
    """Gradients of the mean squared error with respect to every parameter."""
    T, nout = out.shape
    g = {}
    dout = 2.0 * (out - target) / (T * nout)
    g["hw"] = dout.T @ cache["q"]
    g["hb"] = dout.sum(0)
    dq = dout @ p["hw"]                                       # [T][C]
    valid, nv = cache["valid"], cache["nv"]
    dpool = dq[:, None, :] * valid[:, :, None] / nv[:, None, None]    # [T][S][C]
    a = cache["a3"]
    NS, C, H, W = a.shape
    da = np.broadcast_to(dpool.reshape(NS, C, 1, 1) / (H * W), a.shape).copy()
    for l in range(3, -1, -1):
        dz = da * (cache[f"z{l}"] > 0)
        ain = cache[f"a{l - 1}"] if l > 0 else cache["in"]
        Ci = ain.shape[1]
        ap = np.zeros((NS, Ci, H + 2, W + 2))
        ap[:, :, 1:-1, 1:-1] = ain
        gw = np.zeros_like(p[f"w{l}"])
        for dy in range(3):
            for dx in range(3):
                gw[:, :, dy, dx] = np.einsum("nohw,nchw->oc", dz, ap[:, :, dy:dy + H, dx:dx + W])
        g[f"w{l}"] = gw
        g[f"b{l}"] = dz.sum(axis=(0, 2, 3))
        if l > 0:
            dap = np.zeros((NS, Ci, H + 2, W + 2))
            w = p[f"w{l}"]
            for dy in range(3):
                for dx in range(3):
                    dap[:, :, dy:dy + H, dx:dx + W] += np.einsum("nohw,oc->nchw", dz, w[:, :, dy, dx])
            da = dap[:, :, 1:-1, 1:-1]
    return g


def adam_step(p, g, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state holds m, v and the step count t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] -= lr * mh / (np.sqrt(vh) + eps)


# ------------------------------------------------------- fallback decision
def background_given_kernel(stamp, ref, ref_var, ref_mask, sci, sci_var, sci_mask, h):
    """bg = sum w (S - K (x) R) / sum w over the fit set, for one constant stamp."""
    M = core.convolve(ref, stamp)
    phi = core.fit_set(ref_mask, sci_mask, ref_var, sci_var, h)
    w = np.where(phi, 1.0 / (np.asarray(sci_var, np.float64) + ref_var + (~phi)), 0.0)
    r = np.where(phi, np.asarray(sci, np.float64) - M, 0.0)
    return float((w * r).sum() / w.sum())


def accept(chi2_surrogate, dof_surrogate, chi2_plain, dof_plain, factor=1.02):
    """The surrogate is kept where its chi^2/dof is within factor of the plain fit's."""
    return (chi2_surrogate / dof_surrogate) <= factor * (chi2_plain / dof_plain)


def select_per_tile(kernel_coeffs, plain_coeffs, plain_chi2, plain_n, ref, ref_var, ref_mask,
                    sci, sci_var, sci_mask, spec, factor=1.02):
    """Per tile of a PER_TILE constant-kernel spec: the weighted least-squares
    background given the surrogate's kernel (bg = argmin sum w (D0 - bg)^2 over
    the tile's fit set, D0 the difference with zero background), its chi^2 on
    n - 1 degrees of freedom, and the acceptance rule against the plain fit's
    chi^2/(n - n_unknowns).  Returns (coeffs [n][nb + 1], chi2_dof [n],
    accepted [n])."""
    kc = np.asarray(kernel_coeffs, np.float64)
    n, nb = kc.shape
    co0 = np.concatenate([kc, np.zeros((n, 1))], 1)
    stamps, _ = core.expand_kernel(co0, spec)
    D0, _, dmask, _, _ = core.subtract(stamps, np.zeros((n, 1)), ref, ref_var, ref_mask, sci,
                                       sci_var, sci_mask, spec)
    phi = core.fit_set(ref_mask, sci_mask, ref_var, sci_var, spec.half_width)
    with np.errstate(all="ignore"):
        w = np.where(phi, 1.0 / (np.asarray(sci_var, np.float64) + ref_var), 0.0)
    H, W = D0.shape
    out = np.zeros((n, nb + 1))
    rs = np.zeros(n)
    acc = np.zeros(n, bool)
    for t, (x0, x1, y0, y1) in enumerate(core._solve_regions(spec, W, H)):
        sel = phi[y0:y1, x0:x1]
        wt = w[y0:y1, x0:x1][sel]
        d = D0[y0:y1, x0:x1][sel]
        bg = float((wt * d).sum() / wt.sum())
        chi2 = float((wt * (d - bg) ** 2).sum())
        rs[t] = chi2 / (sel.sum() - 1)
        acc[t] = accept(chi2, sel.sum() - 1, plain_chi2[t], plain_n[t] - (nb + 1), factor)
        out[t] = np.r_[kc[t], bg] if acc[t] else plain_coeffs[t]
    return out, rs, acc
