"""Device-side difference-imaging pipeline built from the libargus calls.

Holds the buffers of one camera (masters, reference, scratch planes) in HBM
and runs calibrate -> (coadd) -> fit -> expand -> subtract -> detect on the
current torch stream.  Marshalling only; every step is a HIP kernel.
"""
from __future__ import annotations

import numpy as np

from . import argus


class Pipeline:
    def __init__(self, ctx: argus.Context, W: int, H: int, spec: argus.KernelSpec,
                 psf: np.ndarray, threshold: float = 5.0, capacity: int = 65536,
                 gain: float = 1.0, read_noise: float = 1.7, sat_adu: int = 65535,
                 kappa: float = 3.0, max_iter: int = 5, device: str = "cuda"):
        import torch
        self.torch = torch
        self.ctx, self.W, self.H, self.spec = ctx, W, H, spec
        self.gain, self.read_noise, self.sat_adu = gain, read_noise, sat_adu
        self.kappa, self.max_iter, self.threshold = kappa, max_iter, threshold
        self.n, self.n_solves = argus.kernel_dims(spec)
        dev = torch.device(device)
        f32 = dict(dtype=torch.float32, device=dev)
        u8 = dict(dtype=torch.uint8, device=dev)
        nP = (spec.spatial_degree + 1) * (spec.spatial_degree + 2) // 2
        nPb = (spec.bg_degree + 1) * (spec.bg_degree + 2) // 2
        K = 2 * spec.half_width + 1
        self.sci = torch.empty((H, W), **f32)
        self.sci_var = torch.empty((H, W), **f32)
        self.sci_mask = torch.empty((H, W), **u8)
        self.ref = torch.empty((H, W), **f32)
        self.ref_var = torch.empty((H, W), **f32)
        self.ref_mask = torch.empty((H, W), **u8)
        self.n_used = torch.empty((H, W), **u8)
        self.diff = torch.empty((H, W), **f32)
        self.diff_var = torch.empty((H, W), **f32)
        self.diff_mask = torch.empty((H, W), **u8)
        self.snr = torch.empty((H, W), **f32)
        self.det_mask = torch.empty((H, W), **u8)
        self.coeffs = torch.empty((self.n_solves, self.n), dtype=torch.float64, device=dev)
        self.n_fit = torch.empty(self.n_solves, dtype=torch.int64, device=dev)
        self.status = torch.empty(self.n_solves, dtype=torch.int32, device=dev)
        self.stamps = torch.empty((self.n_solves, nP, K, K), **f32)
        self.bg = torch.empty((self.n_solves, nPb), **f32)
        self.chi2 = torch.empty(self.n_solves, dtype=torch.float64, device=dev)
        self.n_chi2 = torch.empty(self.n_solves, dtype=torch.int64, device=dev)
        self.capacity = capacity
        self.cands = torch.empty(capacity * argus.CANDIDATE_DTYPE.itemsize, **u8)
        self.n_cands = torch.zeros(1, dtype=torch.int32, device=dev)
        self.psf = torch.as_tensor(np.asarray(psf, np.float32), device=dev).contiguous()
        self.psf_half = (self.psf.shape[0] - 1) // 2
        self._cal_scratch = []

    def set_masters(self, dark, flat, bpm):
        t = self.torch
        self.dark = t.as_tensor(np.asarray(dark, np.float32)).cuda()
        self.flat = t.as_tensor(np.asarray(flat, np.float32)).cuda()
        self.bpm = None if bpm is None else t.as_tensor(np.asarray(bpm, np.uint8)).cuda()

    def calibrate(self, raw, cal, var, mask):
        self.ctx.calibrate(raw, self.dark, self.flat, self.bpm, self.gain, self.read_noise,
                           self.sat_adu, cal, var, mask)

    def build_reference(self, raws, fused: bool = True):
        """Calibrate the raw reference frames and coadd them: in one fused
        call (default), or by calibrating each frame into scratch planes and
        coadding those (bit-identical results)."""
        if fused:
            self.ctx.calibrate_coadd(raws, self.dark, self.flat, self.bpm, self.gain,
                                     self.read_noise, self.sat_adu, self.kappa, self.max_iter,
                                     self.ref, self.ref_var, self.ref_mask, self.n_used)
            return
        t = self.torch
        while len(self._cal_scratch) < len(raws):
            self._cal_scratch.append((t.empty_like(self.ref), t.empty_like(self.ref_var),
                                      t.empty_like(self.ref_mask)))
        for raw, (c, v, m) in zip(raws, self._cal_scratch):
            self.calibrate(raw, c, v, m)
        sc = self._cal_scratch[:len(raws)]
        self.ctx.coadd([c for c, _, _ in sc], [v for _, v, _ in sc], [m for _, _, m in sc],
                       self.kappa, self.max_iter, self.ref, self.ref_var, self.ref_mask,
                       self.n_used)

    def difference(self, sci_raw):
        """Calibrate the science frame, fit, expand, subtract and detect."""
        self.calibrate(sci_raw, self.sci, self.sci_var, self.sci_mask)
        self.fit()
        self.subtract()
        self.detect()

    def fit(self):
        self.ctx.fit_kernel(self.spec, self.ref, self.ref_var, self.ref_mask, self.sci,
                            self.sci_var, self.sci_mask, self.coeffs, self.n_fit, self.status)
        self.ctx.expand_kernel(self.spec, self.coeffs, self.stamps, self.bg)

    def subtract(self):
        self.ctx.subtract(self.spec, self.stamps, self.bg, self.ref, self.ref_var,
                          self.ref_mask, self.sci, self.sci_var, self.sci_mask, self.diff,
                          self.diff_var, self.diff_mask, self.chi2, self.n_chi2)

    def detect(self):
        self.ctx.detect(self.diff, self.diff_var, self.diff_mask, self.threshold, self.psf,
                        self.psf_half, self.snr, self.det_mask, self.cands, self.capacity,
                        self.n_cands)

    def candidates(self) -> np.ndarray:
        n = min(int(self.n_cands.item()), self.capacity)
        raw = self.cands[: n * argus.CANDIDATE_DTYPE.itemsize].cpu().numpy()
        return raw.view(argus.CANDIDATE_DTYPE)
