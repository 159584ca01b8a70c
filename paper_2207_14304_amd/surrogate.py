"""Learned kernel surrogate around the plain per-tile fit.

Training pairs come from the plain least-squares fit: a frame pair is cut
into tiles, each tile's fit (constant kernel, constant background) gives the
31 kernel coefficients the network learns to predict from the tile's paired
star stamps.  At inference the network's kernel is judged tile by tile with
the fit's own statistic: given the predicted kernel the background is the
weighted least-squares value, and the tile keeps the prediction only where
its chi^2/dof is within a factor (1.02) of the plain fit's; elsewhere the
plain fit is used.

Host orchestration only: every step is a libargus call (stamp extraction,
CNN forward/backward/Adam, kernel expansion, subtraction, acceptance);
torch supplies device memory and streams, synth_torch the seeded frames.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import argus, synth, synth_torch
from .synth import READ_NOISE_E

TILES = 4
HALF = 7
NB = 31
SNR_MIN = 30.0


def spec(tiles=TILES, half=HALF):
    return argus.make_spec(half_width=half, tiles_x=tiles, tiles_y=tiles,
                           mode=argus.FIT_PER_TILE)


@dataclass
class Conditions:
    """Observing conditions of one synthetic frame pair: reference and science
    FWHM (px), science ellipticity and position angle, sky (e-), flux scale."""
    fwhm_ref: float
    fwhm_sci: float
    ell: float
    theta: float
    sky: float
    scale: float


def draw_conditions(rng) -> Conditions:
    """Seeing 1.5-4.0 px (science broader than the reference by 1.1-1.6x),
    ellipticity 0-0.2 at a random angle, sky 200-3000 e-, scale 0.9-1.1."""
    fr = float(rng.uniform(1.5, 3.0))
    fs = float(min(4.0, fr * rng.uniform(1.1, 1.6)))
    return Conditions(fr, fs, float(rng.uniform(0.0, 0.2)), float(rng.uniform(0, math.pi)),
                      float(rng.uniform(200.0, 3000.0)), float(rng.uniform(0.9, 1.1)))


class Frame:
    """One calibrated frame pair on the device (six planes) and, optionally,
    its noise-free counterpart (expected images with the expected variance)."""

    def __init__(self, ctx, W, H, n_stars, seed, cond: Conditions, noise_free=False):
        import torch
        self.cond = cond
        out = synth_torch.make_pair(W, H, n_stars, seed, cond.fwhm_sci,
                                    ratio=cond.fwhm_ref / cond.fwhm_sci, sky=cond.sky,
                                    scale=cond.scale, ell=cond.ell, theta=cond.theta,
                                    noise_free=noise_free)
        sci_raw, ref_raw = out[0], out[1]
        self.W, self.H = W, H
        dark = torch.zeros((H, W), dtype=torch.float32, device="cuda")
        flat = torch.ones((H, W), dtype=torch.float32, device="cuda")
        planes = []
        for raw in (ref_raw, sci_raw):
            c = torch.empty((H, W), dtype=torch.float32, device="cuda")
            v = torch.empty_like(c)
            m = torch.empty((H, W), dtype=torch.uint8, device="cuda")
            ctx.calibrate(raw, dark, flat, None, 1.0, READ_NOISE_E, 65535, c, v, m)
            planes += [c, v, m]
        self.planes = tuple(planes)
        self.clean = None
        if noise_free:
            sci_e, ref_e = out[4], out[5]
            z = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
            rn2 = READ_NOISE_E ** 2
            self.clean = (ref_e, ref_e + rn2, z, sci_e, sci_e + rn2, z)


class TileFits:
    """Per-tile plain fit of a frame: coefficients, status, chi^2 and fit-set size."""

    def __init__(self, ctx, frame_planes, sp, want_chi2=True):
        import torch
        n, ns = argus.kernel_dims(sp)
        H, W = frame_planes[0].shape
        self.coeffs = torch.empty((ns, n), dtype=torch.float64, device="cuda")
        self.n_fit = torch.empty(ns, dtype=torch.int64, device="cuda")
        self.status = torch.empty(ns, dtype=torch.int32, device="cuda")
        ctx.fit_kernel(sp, *frame_planes, self.coeffs, self.n_fit, self.status)
        self.chi2 = self.n_chi2 = None
        if want_chi2:
            K = 2 * sp.half_width + 1
            st = torch.empty((ns, 1, K, K), dtype=torch.float32, device="cuda")
            bg = torch.empty((ns, 1), dtype=torch.float32, device="cuda")
            ctx.expand_kernel(sp, self.coeffs, st, bg)
            D = torch.empty((H, W), dtype=torch.float32, device="cuda")
            V = torch.empty_like(D)
            M = torch.empty((H, W), dtype=torch.uint8, device="cuda")
            self.chi2 = torch.empty(ns, dtype=torch.float64, device="cuda")
            self.n_chi2 = torch.empty(ns, dtype=torch.int64, device="cuda")
            ctx.subtract(sp, st, bg, *frame_planes, D, V, M, self.chi2, self.n_chi2)


def extract(ctx, frame_planes, tiles=TILES, snr_min=SNR_MIN):
    import torch
    T = tiles * tiles
    X = torch.empty((T, argus.CNN_STAMPS, argus.CNN_NPX, 2), dtype=torch.bfloat16, device="cuda")
    valid = torch.empty((T, argus.CNN_STAMPS), dtype=torch.uint8, device="cuda")
    ovf = torch.zeros(1, dtype=torch.int32, device="cuda")
    ref, rv, rm, sci, sv, sm = frame_planes
    ctx.extract_stamps(ref, rv, rm, sci, sm, tiles, tiles, snr_min, X, valid, ovf)
    return X, valid, ovf


def build_training_set(ctx, n_frames, seed, W=1024, H=1024, n_stars=(300, 4000), tiles=TILES,
                       noise_free_targets=True, log=None):
    """Samples (X bf16 [N][64][961][2], valid u8 [N][64], target f32 [N][31]) from
    n_frames seeded frame pairs.  The inputs are stamps of the noisy frames; the
    targets are the plain per-tile fit's kernel coefficients, by default of the
    noise-free rendering of the same frames (the fit on noisy frames is biased
    low in amplitude by the reference's noise and scatters from tile to tile,
    so it is a poor target), else of the noisy frames themselves.  Tiles whose
    fit failed or that have no valid stamp are dropped."""
    import torch
    rng = np.random.default_rng(seed)
    sp = spec(tiles)
    Xs, Vs, Ts = [], [], []
    for f in range(n_frames):
        cond = draw_conditions(rng)
        ns = int(rng.integers(n_stars[0], n_stars[1] + 1))
        fr = Frame(ctx, W, H, ns, int(seed * 100003 + f), cond, noise_free=noise_free_targets)
        fits = TileFits(ctx, fr.clean if noise_free_targets else fr.planes, sp, want_chi2=False)
        X, valid, _ = extract(ctx, fr.planes, tiles)
        keep = (fits.status == 0) & (valid.sum(1) > 0)
        Xs.append(X[keep])
        Vs.append(valid[keep])
        Ts.append(fits.coeffs[keep, :NB].float())
        if log and (f + 1) % 500 == 0:
            log(f"training set: {f + 1} of {n_frames} frames")
    return torch.cat(Xs), torch.cat(Vs), torch.cat(Ts)


def standardize(target):
    """Per-coefficient mean and standard deviation of the training targets and
    the standardized targets the network is trained on (so that the squared
    error weighs every coefficient alike)."""
    mu = target.mean(0)
    sd = target.std(0).clamp_min(1e-6)
    return (target - mu) / sd, mu, sd


def fold_standardization(flat, mu, sd):
    """Head weights that output coefficients directly: c = mu + sd (W q + b)."""
    layout, _ = argus.cnn_param_layout()
    sw, shw = layout["hw"]
    sb, _ = layout["hb"]
    out = np.array(flat, np.float32, copy=True)
    mu = np.asarray(mu, np.float64)
    sd = np.asarray(sd, np.float64)
    hw = out[sw].reshape(shw).astype(np.float64)
    out[sw] = (sd[:, None] * hw).reshape(-1)
    out[sb] = mu + sd * out[sb].astype(np.float64)
    return out


def train(cnn: argus.CNN, X, valid, target, epochs, batch, lr, seed=0, log=None):
    """Minibatch Adam on the GPU; returns the per-step loss history (host)."""
    import torch
    N = X.shape[0]
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).cuda()
        for i in range(0, N - batch + 1, batch):
            idx = perm[i:i + batch]
            xb = X.index_select(0, idx).contiguous()
            vb = valid.index_select(0, idx).contiguous()
            tb = target.index_select(0, idx).contiguous()
            cnn.train_step(xb, vb, tb, lr, loss)
            hist.append(loss.clone())
        if log:
            log(f"epoch {ep}: loss {float(hist[-1].item()):.4g}")
    return np.array([float(h.item()) for h in hist])


def init_weights(seed, C=32, cin=2, nout=NB):
    """He-normal convolution weights, zero biases, a small head (flat layout of
    argus_cnn_set_weights)."""
    layout, n = argus.cnn_param_layout(C, cin, nout)
    rng = np.random.default_rng(seed)
    flat = np.zeros(n, np.float32)
    for l in range(4):
        sl, shp = layout[f"w{l}"]
        fan = shp[1] * shp[2]
        flat[sl] = rng.standard_normal(sl.stop - sl.start) * math.sqrt(2.0 / fan)
    sl, shp = layout["hw"]
    flat[sl] = rng.standard_normal(sl.stop - sl.start) * math.sqrt(1.0 / shp[1]) * 0.1
    return flat


class SurrogatePath:
    """Per-frame surrogate path: stamps -> CNN -> kernel -> subtraction with zero
    background -> background, chi^2/dof and acceptance per tile -> final
    coefficients (the surrogate's where accepted, else the plain fit's)."""

    def __init__(self, ctx, cnn: argus.CNN, W, H, tiles=TILES, half=HALF, factor=1.02):
        import torch
        self.ctx, self.cnn, self.factor = ctx, cnn, factor
        self.sp = spec(tiles, half)
        n, ns = argus.kernel_dims(self.sp)
        self.n, self.ns = n, ns
        K = 2 * half + 1
        f64 = dict(dtype=torch.float64, device="cuda")
        self.out = torch.empty((ns, NB), dtype=torch.float32, device="cuda")
        self.sco = torch.empty((ns, n), **f64)
        self.stamps = torch.empty((ns, 1, K, K), dtype=torch.float32, device="cuda")
        self.bg = torch.empty((ns, 1), dtype=torch.float32, device="cuda")
        self.D = torch.empty((H, W), dtype=torch.float32, device="cuda")
        self.V = torch.empty_like(self.D)
        self.M = torch.empty((H, W), dtype=torch.uint8, device="cuda")
        self.c0 = torch.empty(ns, **f64)
        self.n0 = torch.empty(ns, dtype=torch.int64, device="cuda")
        self.swd = torch.empty(ns, **f64)
        self.sw = torch.empty(ns, **f64)
        self.coeffs = torch.empty((ns, n), **f64)
        self.chi2_dof = torch.empty(ns, **f64)
        self.accepted = torch.empty(ns, dtype=torch.int32, device="cuda")

    def predict(self, planes):
        """Network kernel per tile and its zero-background subtraction sums."""
        X, valid, _ = extract(self.ctx, planes, self.sp.tiles_x)
        self.cnn.forward(X, valid, self.out)
        self.ctx.surrogate_coeffs(self.out, self.sco)
        self.ctx.expand_kernel(self.sp, self.sco, self.stamps, self.bg)
        self.ctx.subtract(self.sp, self.stamps, self.bg, *planes, self.D, self.V, self.M,
                          self.c0, self.n0, self.swd, self.sw)

    def select(self, plain: TileFits | None = None, ref_chi2_dof=0.0):
        if plain is not None:
            self.ctx.surrogate_select(self.sco, self.c0, self.n0, self.swd, self.sw, self.coeffs,
                                      self.chi2_dof, self.accepted, plain_coeffs=plain.coeffs,
                                      plain_chi2=plain.chi2, plain_n=plain.n_chi2,
                                      factor=self.factor)
        else:
            self.ctx.surrogate_select(self.sco, self.c0, self.n0, self.swd, self.sw, self.coeffs,
                                      self.chi2_dof, self.accepted, ref_chi2_dof=ref_chi2_dof,
                                      factor=self.factor)

    def subtract_final(self, planes, chi2=None, n_chi2=None):
        self.ctx.expand_kernel(self.sp, self.coeffs, self.stamps, self.bg)
        self.ctx.subtract(self.sp, self.stamps, self.bg, *planes, self.D, self.V, self.M,
                          chi2, n_chi2)


def kernel_error(coeffs, truth, B, psf=None):
    """||K - K_true|| / ||K_true|| per tile, K = sum_k a_k B_k (host arrays);
    with psf, of the kernels convolved with it (the error in the model of a
    star, where the fit's poorly constrained high frequencies drop out)."""
    K = np.tensordot(np.asarray(coeffs)[:, :NB], B, 1)
    Kt = np.tensordot(np.asarray(truth)[:, :NB], B, 1)
    if psf is not None:
        from scipy import signal
        K = np.stack([signal.convolve2d(k, psf) for k in K])
        Kt = np.stack([signal.convolve2d(k, psf) for k in Kt])
    return np.linalg.norm((K - Kt).reshape(len(K), -1), axis=1) / \
        np.linalg.norm(Kt.reshape(len(K), -1), axis=1)


def basis_stamps(ctx, half=HALF):
    """The normalised basis B[k][v][u] as the library expands it (host array)."""
    import torch
    sp = argus.make_spec(half_width=half, tiles_x=NB, tiles_y=1, mode=argus.FIT_PER_TILE)
    K = 2 * half + 1
    co = torch.zeros((NB, NB + 1), dtype=torch.float64, device="cuda")
    co[:, :NB] = torch.eye(NB, dtype=torch.float64, device="cuda")
    st = torch.empty((NB, 1, K, K), dtype=torch.float32, device="cuda")
    bg = torch.empty((NB, 1), dtype=torch.float32, device="cuda")
    ctx.expand_kernel(sp, co, st, bg)
    return st[:, 0].double().cpu().numpy()


def evaluate(ctx, path: "SurrogatePath", frames, B):
    """Per tile of every frame: kernel errors of the plain fit and of the
    network against the fit on the noise-free frames, the acceptance, and the
    chi^2/dof of the plain fit and of the final (accepted or fallback) kernel;
    status is nonzero where the plain fit or the noise-free fit failed."""
    import torch
    sp = path.sp
    rows = []
    c2 = torch.empty(path.ns, dtype=torch.float64, device="cuda")
    n2 = torch.empty(path.ns, dtype=torch.int64, device="cuda")
    for fr in frames:
        plain = TileFits(ctx, fr.planes, sp)
        truth = TileFits(ctx, fr.clean, sp, want_chi2=False)
        path.predict(fr.planes)
        path.select(plain)
        path.subtract_final(fr.planes, c2, n2)
        co_p = plain.coeffs.cpu().numpy()
        co_s = path.sco.cpu().numpy()
        co_t = truth.coeffs.cpu().numpy()
        e_p = kernel_error(co_p, co_t, B)
        e_s = kernel_error(co_s, co_t, B)
        psf = synth.psf_image(10, fr.cond.fwhm_ref)
        m_p = kernel_error(co_p, co_t, B, psf)
        m_s = kernel_error(co_s, co_t, B, psf)
        rp = (plain.chi2 / (plain.n_chi2 - (NB + 1))).cpu().numpy()
        rf = (c2 / n2.clamp_min(1)).cpu().numpy()
        acc = path.accepted.cpu().numpy()
        st = plain.status.cpu().numpy()
        stt = truth.status.cpu().numpy()
        for t in range(path.ns):
            rows.append(dict(err_plain=float(e_p[t]), err_sur=float(e_s[t]),
                             model_err_plain=float(m_p[t]), model_err_sur=float(m_s[t]),
                             accepted=int(acc[t]), chi2dof_plain=float(rp[t]),
                             chi2dof_final=float(rf[t]),
                             status=int(st[t]) if st[t] != 0 else int(stt[t]),
                             plain_status=int(st[t]), truth_status=int(stt[t])))
    return rows
