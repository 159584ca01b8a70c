"""Python binding of libargus (ctypes).

Argument marshalling only: every step runs in the HIP library.  Tensors are
torch device tensors used for their memory and stream; the calls enqueue on
``torch.cuda.current_stream()`` and do not synchronise.  There is no CPU
fallback: loading fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libargus.so")

OK, EINVAL, ESHAPE, ENOMEM, EHIP, EBUSY = 0, -1, -2, -3, -4, -5
ESINGULAR, ETOOFEW = -20, -21
BAD, SAT, EDGE, NODATA, FOOT, DET, CAND = 0x01, 0x02, 0x04, 0x08, 0x10, 0x20, 0x40
FIT_GLOBAL, FIT_PER_TILE = 0, 1
FP32, BF16X3, FP64 = 0, 1, 2

# every symbol declared in include/argus.h
SYMBOLS = ("argus_ctx_create", "argus_ctx_destroy", "argus_ctx_set_stream", "argus_last_error",
           "argus_ctx_set_timing", "argus_kernel_time_ms", "argus_calibrate", "argus_coadd",
           "argus_calibrate_coadd",
           "argus_kernel_dims", "argus_fit_kernel", "argus_expand_kernel", "argus_subtract",
           "argus_subtract_noalloc", "argus_detect", "argus_batch_plan", "argus_batch_run", "argus_batch_info",
           "argus_batch_destroy", "argus_batch_tuning", "argus_batch_candidate", "argus_ctx_set_tune_cache", "argus_cnn_create", "argus_cnn_destroy",
           "argus_cnn_n_params", "argus_cnn_set_weights", "argus_cnn_get_weights",
           "argus_cnn_get_grads", "argus_cnn_forward", "argus_cnn_train_step",
           "argus_surrogate_coeffs", "argus_surrogate_select", "argus_extract_stamps",
           "argus_background", "argus_detect_sources", "argus_coadd_matched",
           "argus_healpix_tiles", "argus_resample_healpix", "argus_zogy")


class Dims(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("pitch", C.c_int64)]


class Wcs(C.Structure):
    """argus_wcs: gnomonic frame geometry (degrees; cd row-major)."""
    _fields_ = [("ra0", C.c_double), ("dec0", C.c_double), ("crpix1", C.c_double),
                ("crpix2", C.c_double), ("cd", C.c_double * 4)]


def make_wcs(ra0, dec0, crpix1, crpix2, cd) -> Wcs:
    w = Wcs()
    w.ra0, w.dec0, w.crpix1, w.crpix2 = float(ra0), float(dec0), float(crpix1), float(crpix2)
    for i, v in enumerate(np.asarray(cd, np.float64).ravel()):
        w.cd[i] = float(v)
    return w


def healpix_tiles(wcs: Wcs, width: int, height: int, nside: int = 256, step: int = 32):
    """argus_healpix_tiles: the (face, I, J) tiles the frame falls in, [n][3] int32."""
    lib = load()
    cap = 4096
    while True:
        buf = np.zeros((cap, 3), np.int32)
        n = C.c_int()
        rc = lib.argus_healpix_tiles(C.byref(wcs), int(width), int(height), int(nside), int(step),
                                     buf.ctypes.data_as(C.c_void_p), cap, C.byref(n))
        if rc:
            raise ArgusError(rc, "argus_healpix_tiles failed")
        if n.value <= cap:
            return buf[: n.value].copy()
        cap = n.value


class KernelSpec(C.Structure):
    _fields_ = [("n_gauss", C.c_int32), ("sigma", C.c_double * 4), ("degree", C.c_int32 * 4),
                ("half_width", C.c_int32), ("spatial_degree", C.c_int32),
                ("bg_degree", C.c_int32), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("mode", C.c_int32), ("precision", C.c_int32)]


class Cutout(C.Structure):
    _fields_ = [("frame", C.c_int32), ("x0", C.c_int32), ("y0", C.c_int32), ("side", C.c_int32),
                ("out_offset", C.c_int64)]


class Frame(C.Structure):
    _fields_ = [("ref", C.c_void_p), ("ref_var", C.c_void_p), ("ref_mask", C.c_void_p),
                ("sci", C.c_void_p), ("sci_var", C.c_void_p), ("sci_mask", C.c_void_p),
                ("width", C.c_int32), ("height", C.c_int32), ("pitch", C.c_int64)]


SOURCE_DTYPE = np.dtype([("x", np.int32), ("y", np.int32), ("xc", np.float32), ("yc", np.float32),
                         ("snr", np.float32), ("flux", np.float32), ("flux_err", np.float32)])
CANDIDATE_DTYPE = np.dtype([("x", np.int32), ("y", np.int32), ("snr", np.float32),
                            ("flux", np.float32), ("flux_err", np.float32)])


def make_spec(sigmas=(0.7, 1.5, 3.0), degrees=(4, 3, 2), half_width=7, spatial_degree=0,
              bg_degree=0, tiles_x=1, tiles_y=1, mode=FIT_GLOBAL, precision=FP32) -> KernelSpec:
    s = KernelSpec()
    s.n_gauss = len(sigmas)
    for i, (sg, d) in enumerate(zip(sigmas, degrees)):
        s.sigma[i] = float(sg)
        s.degree[i] = int(d)
    s.half_width = half_width
    s.spatial_degree = spatial_degree
    s.bg_degree = bg_degree
    s.tiles_x, s.tiles_y = tiles_x, tiles_y
    s.mode, s.precision = mode, precision
    return s


_lib = None


def load(path: str = LIB_PATH):
    """Load libargus.so and declare the signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libargus.so not built at {path}; run python -m paper_2207_14304_amd.build")
    lib = C.CDLL(path)
    vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    lib.argus_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
    lib.argus_ctx_destroy.argtypes = [vp]
    lib.argus_ctx_destroy.restype = None
    lib.argus_ctx_set_stream.argtypes = [vp, vp]
    lib.argus_last_error.argtypes = [vp]
    lib.argus_last_error.restype = C.c_char_p
    lib.argus_ctx_set_timing.argtypes = [vp, C.c_int]
    lib.argus_kernel_time_ms.argtypes = [vp, C.c_char_p]
    lib.argus_kernel_time_ms.restype = f32
    lib.argus_calibrate.argtypes = [vp, Dims, vp, vp, vp, vp, f32, f32, C.c_uint16, vp, vp, vp]
    lib.argus_coadd.argtypes = [vp, Dims, C.c_int, vp, vp, vp, f32, C.c_int, vp, vp, vp, vp]
    lib.argus_calibrate_coadd.argtypes = [vp, Dims, C.c_int, vp, vp, vp, vp, f32, f32, C.c_uint16,
                                          f32, C.c_int, vp, vp, vp, vp]
    lib.argus_kernel_dims.argtypes = [C.POINTER(KernelSpec), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.argus_fit_kernel.argtypes = [vp, Dims, C.POINTER(KernelSpec)] + [vp] * 10
    lib.argus_expand_kernel.argtypes = [vp, C.POINTER(KernelSpec), vp, vp, vp]
    lib.argus_subtract.argtypes = [vp, Dims, C.POINTER(KernelSpec)] + [vp] * 15
    lib.argus_subtract_noalloc.argtypes = [vp, Dims, C.POINTER(KernelSpec)] + [vp] * 15
    lib.argus_background.argtypes = [vp, Dims, vp, vp, C.c_int, vp, vp, vp]
    d64 = C.c_double
    lib.argus_zogy.argtypes = [vp, Dims, vp, vp, vp, vp, vp, C.c_int, C.c_int, vp, vp, C.c_int,
                               d64, d64, d64, d64, vp, vp, vp, vp, vp]
    lib.argus_healpix_tiles.argtypes = [C.POINTER(Wcs), C.c_int, C.c_int, C.c_int, C.c_int, vp,
                                        C.c_int, C.POINTER(C.c_int)]
    lib.argus_resample_healpix.argtypes = [vp, Dims, vp, vp, vp, C.POINTER(Wcs), C.c_int, C.c_int,
                                           vp, C.c_int, vp, vp, vp]
    lib.argus_coadd_matched.argtypes = [vp, Dims, C.c_int, vp, vp, vp, vp, C.c_int, vp, C.c_int,
                                        vp, vp, vp, vp]
    lib.argus_detect_sources.argtypes = [vp, Dims, vp, vp, vp, vp, C.c_int, f32, vp, C.c_int, vp,
                                         vp, vp, C.c_int32, vp]
    lib.argus_detect.argtypes = [vp, Dims, vp, vp, vp, f32, vp, C.c_int, vp, vp, vp, i32, vp]
    lib.argus_batch_plan.argtypes = [vp, C.POINTER(KernelSpec), C.POINTER(Cutout), C.c_int,
                                     C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int,
                                     C.POINTER(vp)]
    lib.argus_batch_run.argtypes = [vp, vp, C.POINTER(Frame), f32] + [vp] * 9
    lib.argus_batch_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(f32), C.POINTER(C.c_int)]
    lib.argus_batch_tuning.argtypes = [vp, C.POINTER(f32), C.c_int, C.POINTER(C.c_int),
                                       C.POINTER(C.c_int)]
    lib.argus_batch_candidate.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.argus_ctx_set_tune_cache.argtypes = [vp, C.c_char_p]
    lib.argus_batch_destroy.argtypes = [vp]
    lib.argus_batch_destroy.restype = None
    lib.argus_cnn_create.argtypes = [vp, C.c_int, C.POINTER(vp)]
    lib.argus_cnn_destroy.argtypes = [vp]
    lib.argus_cnn_destroy.restype = None
    lib.argus_cnn_n_params.argtypes = [vp]
    lib.argus_cnn_set_weights.argtypes = [vp, vp, vp]
    lib.argus_cnn_get_weights.argtypes = [vp, vp, vp]
    lib.argus_cnn_get_grads.argtypes = [vp, vp, vp]
    lib.argus_cnn_forward.argtypes = [vp, vp, vp, vp, C.c_int, vp]
    lib.argus_cnn_train_step.argtypes = [vp, vp, vp, vp, vp, C.c_int, f32, vp]
    lib.argus_surrogate_coeffs.argtypes = [vp, C.c_int, C.c_int, vp, vp]
    lib.argus_surrogate_select.argtypes = [vp, C.c_int, C.c_int] + [vp] * 8 + \
        [C.c_double, C.c_double, vp, vp, vp]
    lib.argus_extract_stamps.argtypes = [vp, Dims, vp, vp, vp, vp, vp, C.c_int, C.c_int, f32,
                                         C.c_int, C.c_int, vp, vp, vp]
    for name in SYMBOLS:
        if name not in ("argus_ctx_destroy", "argus_last_error", "argus_kernel_time_ms",
                        "argus_batch_destroy", "argus_cnn_destroy"):
            getattr(lib, name).restype = C.c_int
    _ = (i64,)
    _lib = lib
    return lib


class ArgusError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"argus error {code}: {msg}")
        self.code = code


def batch_candidate(index: int):
    """(subtraction tile rows, workgroups per CU) of autotuner candidate ``index``."""
    lib = load()
    t, w = C.c_int(), C.c_int()
    rc = lib.argus_batch_candidate(index, C.byref(t), C.byref(w))
    if rc:
        raise ArgusError(rc, f"no batch candidate {index}")
    return t.value, w.value


def kernel_dims(spec: KernelSpec):
    lib = load()
    n, s = C.c_int(), C.c_int()
    rc = lib.argus_kernel_dims(C.byref(spec), C.byref(n), C.byref(s))
    if rc:
        raise ArgusError(rc, "bad kernel spec")
    return n.value, s.value


def _ptr(t, dtype=None):
    """Device address of a torch tensor (or 0 for None), checking dtype."""
    if t is None:
        return None
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise TypeError("expected a device tensor")
    return t.data_ptr()


def _dims(t):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("images are 2-D, row-major with unit column stride")
    return Dims(t.shape[1], t.shape[0], t.stride(0))


class Context:
    """An argus_ctx bound to the current torch stream of ``device``."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.lib = load()
        self.device = device
        h = C.c_void_p()
        rc = self.lib.argus_ctx_create(device, C.byref(h))
        if rc:
            raise ArgusError(rc, "argus_ctx_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.argus_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind(self):
        s = self._torch.cuda.current_stream(self.device).cuda_stream
        self.lib.argus_ctx_set_stream(self.h, C.c_void_p(s))

    def _check(self, rc):
        if rc:
            raise ArgusError(rc, self.lib.argus_last_error(self.h).decode())

    def set_timing(self, on: bool):
        self._check(self.lib.argus_ctx_set_timing(self.h, int(on)))

    def set_tune_cache(self, path):
        """Read the autotuner's JSON-lines cache at ``path`` and append new
        outcomes to it (None: in memory only)."""
        self._check(self.lib.argus_ctx_set_tune_cache(self.h, None if path is None else
                                                      str(path).encode()))

    def kernel_time_ms(self, name: str) -> float:
        return float(self.lib.argus_kernel_time_ms(self.h, name.encode()))

    # ---- calls ------------------------------------------------------------
    def calibrate(self, raw, dark, flat, bpm, gain, read_noise, sat_adu, cal, var, mask):
        torch = self._torch
        self._bind()
        self._check(self.lib.argus_calibrate(
            self.h, _dims(raw), _ptr(raw, torch.uint16), _ptr(dark, torch.float32),
            _ptr(flat, torch.float32), _ptr(bpm, torch.uint8), float(gain), float(read_noise),
            int(sat_adu), _ptr(cal, torch.float32), _ptr(var, torch.float32),
            _ptr(mask, torch.uint8)))

    def coadd(self, cals, vars_, masks, kappa, max_iter, ref, ref_var, ref_mask, n_used=None):
        torch = self._torch
        self._bind()
        n = len(cals)
        P = C.c_void_p * n
        pc = P(*[_ptr(c, torch.float32) for c in cals])
        pv = P(*[_ptr(v, torch.float32) for v in vars_])
        pm = P(*[_ptr(m, torch.uint8) for m in masks])
        self._check(self.lib.argus_coadd(
            self.h, _dims(cals[0]), n, pc, pv, pm, float(kappa), int(max_iter),
            _ptr(ref, torch.float32), _ptr(ref_var, torch.float32), _ptr(ref_mask, torch.uint8),
            _ptr(n_used, torch.uint8)))

    def calibrate_coadd(self, raws, dark, flat, bpm, gain, read_noise, sat_adu, kappa, max_iter,
                        ref, ref_var, ref_mask, n_used=None):
        torch = self._torch
        self._bind()
        n = len(raws)
        pr = (C.c_void_p * n)(*[_ptr(r, torch.uint16) for r in raws])
        self._check(self.lib.argus_calibrate_coadd(
            self.h, _dims(raws[0]), n, pr, _ptr(dark, torch.float32), _ptr(flat, torch.float32),
            _ptr(bpm, torch.uint8), float(gain), float(read_noise), int(sat_adu), float(kappa),
            int(max_iter), _ptr(ref, torch.float32), _ptr(ref_var, torch.float32),
            _ptr(ref_mask, torch.uint8), _ptr(n_used, torch.uint8)))

    def fit_kernel(self, spec, ref, ref_var, ref_mask, sci, sci_var, sci_mask, coeffs, n_fit,
                   status, chi2=None):
        torch = self._torch
        self._bind()
        self._check(self.lib.argus_fit_kernel(
            self.h, _dims(ref), C.byref(spec), _ptr(ref, torch.float32),
            _ptr(ref_var, torch.float32), _ptr(ref_mask, torch.uint8), _ptr(sci, torch.float32),
            _ptr(sci_var, torch.float32), _ptr(sci_mask, torch.uint8),
            _ptr(coeffs, torch.float64), _ptr(chi2, torch.float64), _ptr(n_fit, torch.int64),
            _ptr(status, torch.int32)))

    def expand_kernel(self, spec, coeffs, stamps, bg):
        torch = self._torch
        self._bind()
        self._check(self.lib.argus_expand_kernel(
            self.h, C.byref(spec), _ptr(coeffs, torch.float64), _ptr(stamps, torch.float32),
            _ptr(bg, torch.float32)))

    def subtract(self, spec, stamps, bg, ref, ref_var, ref_mask, sci, sci_var, sci_mask, diff,
                 diff_var, diff_mask, chi2=None, n_chi2=None, sum_wd=None, sum_w=None,
                 noalloc=False):
        """argus_subtract, or with noalloc=True argus_subtract_noalloc (same
        results; partial sums in the library's fixed scratch, no allocation)."""
        torch = self._torch
        self._bind()
        fn = self.lib.argus_subtract_noalloc if noalloc else self.lib.argus_subtract
        self._check(fn(
            self.h, _dims(ref), C.byref(spec), _ptr(stamps, torch.float32),
            _ptr(bg, torch.float32), _ptr(ref, torch.float32), _ptr(ref_var, torch.float32),
            _ptr(ref_mask, torch.uint8), _ptr(sci, torch.float32), _ptr(sci_var, torch.float32),
            _ptr(sci_mask, torch.uint8), _ptr(diff, torch.float32),
            _ptr(diff_var, torch.float32), _ptr(diff_mask, torch.uint8),
            _ptr(chi2, torch.float64), _ptr(n_chi2, torch.int64), _ptr(sum_wd, torch.float64),
            _ptr(sum_w, torch.float64)))

    def detect(self, diff, diff_var, diff_mask, threshold, psf, psf_half, snr, det_mask, cands,
               capacity, n_cands):
        torch = self._torch
        self._bind()
        self._check(self.lib.argus_detect(
            self.h, _dims(diff), _ptr(diff, torch.float32), _ptr(diff_var, torch.float32),
            _ptr(diff_mask, torch.uint8), float(threshold), _ptr(psf, torch.float32),
            int(psf_half), _ptr(snr, torch.float32), _ptr(det_mask, torch.uint8),
            _ptr(cands, torch.uint8), int(capacity), _ptr(n_cands, torch.int32)))


def _background(self, cal, mask, box, grid, levels=None, bg_map=None):
    """argus_background: filtered cell grid (and optionally the raw levels and
    the full-resolution map) of a calibrated frame."""
    torch = self._torch
    self._bind()
    self._check(self.lib.argus_background(
        self.h, _dims(cal), _ptr(cal, torch.float32), _ptr(mask, torch.uint8), int(box),
        _ptr(levels, torch.float32), _ptr(grid, torch.float32), _ptr(bg_map, torch.float32)))


def _detect_sources(self, cal, var, mask, grid, box, threshold, psf, psf_half, snr, det_mask,
                    sources, capacity, n_sources):
    """argus_detect_sources; sources is a uint8 buffer of capacity * SOURCE_DTYPE.itemsize."""
    torch = self._torch
    self._bind()
    self._check(self.lib.argus_detect_sources(
        self.h, _dims(cal), _ptr(cal, torch.float32), _ptr(var, torch.float32),
        _ptr(mask, torch.uint8), _ptr(grid, torch.float32), int(box), float(threshold),
        _ptr(psf, torch.float32), int(psf_half), _ptr(snr, torch.float32),
        _ptr(det_mask, torch.uint8), _ptr(sources, torch.uint8), int(capacity),
        _ptr(n_sources, torch.int32)))


def _coadd_matched(self, cals, vars_, masks, psf, psf_half, score, score_var, snr=None,
                   grids=None, box=64, scales=None):
    """argus_coadd_matched: psf a device f32 [n][2r+1][2r+1] tensor; grids a
    list (entries may be None) of background grids; scales host floats."""
    torch = self._torch
    self._bind()
    n = len(cals)
    arr = C.c_void_p * n
    g = arr(*[_ptr(x, torch.float32) if x is not None else None for x in (grids or [None] * n)])
    sc = (C.c_float * n)(*[float(v) for v in scales]) if scales is not None else None
    self._check(self.lib.argus_coadd_matched(
        self.h, _dims(score), n, arr(*[_ptr(c, torch.float32) for c in cals]),
        arr(*[_ptr(v, torch.float32) for v in vars_]), arr(*[_ptr(m, torch.uint8) for m in masks]),
        g, int(box), _ptr(psf, torch.float32), int(psf_half), sc, _ptr(score, torch.float32),
        _ptr(score_var, torch.float32), _ptr(snr, torch.float32)))


def _resample_healpix(self, cal, var, mask, wcs, nside, m, tiles, out, out_var, out_mask):
    """argus_resample_healpix: tiles a device int32 [n][3] tensor."""
    torch = self._torch
    self._bind()
    if tiles.dtype != torch.int32 or tiles.dim() != 2 or tiles.shape[1] != 3:
        raise ValueError("tiles: int32 [n][3]")
    self._check(self.lib.argus_resample_healpix(
        self.h, _dims(cal), _ptr(cal, torch.float32), _ptr(var, torch.float32),
        _ptr(mask, torch.uint8), C.byref(wcs), int(nside), int(m), _ptr(tiles, torch.int32),
        int(tiles.shape[0]), _ptr(out, torch.float32), _ptr(out_var, torch.float32),
        _ptr(out_mask, torch.uint8)))


def _zogy(self, new, new_mask, ref, ref_mask, origins, L, psf_n, psf_r, psf_half, Fn, Fr, sn, sr,
          D, snr, flux, mask, pd2=None):
    """argus_zogy: origins a device int32 [n][2] tensor (x0, y0 per tile)."""
    torch = self._torch
    self._bind()
    if origins.dtype != torch.int32 or origins.dim() != 2 or origins.shape[1] != 2:
        raise ValueError("origins: int32 [n][2]")
    self._check(self.lib.argus_zogy(
        self.h, _dims(new), _ptr(new, torch.float32), _ptr(new_mask, torch.uint8),
        _ptr(ref, torch.float32), _ptr(ref_mask, torch.uint8), _ptr(origins, torch.int32),
        int(origins.shape[0]), int(L), _ptr(psf_n, torch.float32), _ptr(psf_r, torch.float32),
        int(psf_half), float(Fn), float(Fr), float(sn), float(sr), _ptr(D, torch.float32),
        _ptr(snr, torch.float32), _ptr(flux, torch.float32), _ptr(mask, torch.uint8),
        _ptr(pd2, torch.float64)))


Context.zogy = _zogy
Context.resample_healpix = _resample_healpix
Context.coadd_matched = _coadd_matched
Context.background = _background
Context.detect_sources = _detect_sources


class Batch:
    """A planned batch of cutouts (argus_batch_plan); run with Context.batch_run."""

    def __init__(self, ctx: "Context", spec: KernelSpec, frame, x0, y0, side, widths, heights):
        self.ctx = ctx
        self.spec = spec
        side = np.asarray(side, np.int64)
        self.n = int(side.size)
        self.side = side
        self.offsets = np.concatenate([[0], np.cumsum(side * side)[:-1]]).astype(np.int64)
        self.arena = int((side * side).sum())
        arr = (Cutout * self.n)()
        for i in range(self.n):
            arr[i] = Cutout(int(frame[i]), int(x0[i]), int(y0[i]), int(side[i]),
                            int(self.offsets[i]))
        nf = len(widths)
        w = (C.c_int32 * nf)(*[int(v) for v in widths])
        h = (C.c_int32 * nf)(*[int(v) for v in heights])
        hnd = C.c_void_p()
        ctx._bind()
        ctx._check(ctx.lib.argus_batch_plan(ctx.h, C.byref(spec), arr, self.n, w, h, nf,
                                            C.byref(hnd)))
        self.h = hnd
        self.n_frames = nf

    def info(self):
        c, ms, n = C.c_int(), C.c_float(), C.c_int()
        self.ctx.lib.argus_batch_info(self.h, C.byref(c), C.byref(ms), C.byref(n))
        return c.value, ms.value, n.value

    def tuning(self):
        """(per-candidate times in ms, taken from the tuning cache?)"""
        buf = (C.c_float * 64)()
        n, hit = C.c_int(), C.c_int()
        self.ctx._check(self.ctx.lib.argus_batch_tuning(self.h, buf, 64, C.byref(n), C.byref(hit)))
        return [buf[i] for i in range(min(n.value, 64))], bool(hit.value)

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.argus_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch_run(self, batch: Batch, frames, threshold, diff, diff_var, diff_mask, det_mask,
               coeffs, chi2, n_fit, status, n_cands):
    """frames: list of (ref, ref_var, ref_mask, sci, sci_var, sci_mask) device tensors."""
    torch = self._torch
    self._bind()
    arr = (Frame * len(frames))()
    for i, f in enumerate(frames):
        d = _dims(f[0])
        arr[i] = Frame(_ptr(f[0], torch.float32), _ptr(f[1], torch.float32),
                       _ptr(f[2], torch.uint8), _ptr(f[3], torch.float32),
                       _ptr(f[4], torch.float32), _ptr(f[5], torch.uint8),
                       d.width, d.height, d.pitch)
    self._check(self.lib.argus_batch_run(
        self.h, batch.h, arr, float(threshold), _ptr(diff, torch.float32),
        _ptr(diff_var, torch.float32), _ptr(diff_mask, torch.uint8), _ptr(det_mask, torch.uint8),
        _ptr(coeffs, torch.float64), _ptr(chi2, torch.float64), _ptr(n_fit, torch.int64),
        _ptr(status, torch.int32), _ptr(n_cands, torch.int32)))


Context.batch_run = _batch_run


# ---- learned kernel surrogate ----------------------------------------------
CNN_STAMPS, CNN_HALF, CNN_NPX = 64, 15, 31 * 31


def _surrogate_coeffs(self, cnn_out, coeffs):
    torch = self._torch
    self._bind()
    n, nb = cnn_out.shape
    self._check(self.lib.argus_surrogate_coeffs(self.h, int(n), int(nb),
                                                _ptr(cnn_out, torch.float32),
                                                _ptr(coeffs, torch.float64)))


def _surrogate_select(self, sur_coeffs, chi2_0, n_0, sum_wd, sum_w, coeffs_out, chi2_dof,
                      accepted, plain_coeffs=None, plain_chi2=None, plain_n=None,
                      ref_chi2_dof=0.0, factor=1.02):
    torch = self._torch
    self._bind()
    n, nc = sur_coeffs.shape
    self._check(self.lib.argus_surrogate_select(
        self.h, int(n), int(nc - 1), _ptr(sur_coeffs, torch.float64), _ptr(chi2_0, torch.float64),
        _ptr(n_0, torch.int64), _ptr(sum_wd, torch.float64), _ptr(sum_w, torch.float64),
        _ptr(plain_coeffs, torch.float64), _ptr(plain_chi2, torch.float64),
        _ptr(plain_n, torch.int64), float(ref_chi2_dof), float(factor),
        _ptr(coeffs_out, torch.float64), _ptr(chi2_dof, torch.float64),
        _ptr(accepted, torch.int32)))


def _extract_stamps(self, ref, ref_var, ref_mask, sci, sci_mask, tiles_x, tiles_y, snr_min, X,
                    valid, overflow, stamps_per_tile=CNN_STAMPS, half=CNN_HALF):
    """X: bf16 device tensor [T][S][(2 half+1)^2][2]; valid u8 [T][S]; overflow i32 [1]."""
    torch = self._torch
    self._bind()
    if X.dtype != torch.bfloat16 or not X.is_contiguous():
        raise TypeError("X must be a contiguous bfloat16 tensor")
    self._check(self.lib.argus_extract_stamps(
        self.h, _dims(ref), _ptr(ref, torch.float32), _ptr(ref_var, torch.float32),
        _ptr(ref_mask, torch.uint8), _ptr(sci, torch.float32), _ptr(sci_mask, torch.uint8),
        int(tiles_x), int(tiles_y), float(snr_min), int(stamps_per_tile), int(half),
        X.data_ptr(), _ptr(valid, torch.uint8), _ptr(overflow, torch.int32)))


Context.surrogate_coeffs = _surrogate_coeffs
Context.surrogate_select = _surrogate_select
Context.extract_stamps = _extract_stamps


class CNN:
    """An argus_cnn handle: the surrogate network's parameters, Adam state and
    activation buffers for up to max_tiles tiles of 64 stamp pairs."""

    def __init__(self, ctx: "Context", max_tiles: int):
        self.ctx = ctx
        h = C.c_void_p()
        ctx._bind()
        ctx._check(ctx.lib.argus_cnn_create(ctx.h, int(max_tiles), C.byref(h)))
        self.h = h
        self.max_tiles = int(max_tiles)
        self.n_params = int(ctx.lib.argus_cnn_n_params(h))

    def _host(self, fn, arr=None):
        a = np.empty(self.n_params, np.float32) if arr is None else arr
        self.ctx._bind()
        self.ctx._check(fn(self.ctx.h, self.h, a.ctypes.data))
        return a

    def set_weights(self, params):
        p = np.ascontiguousarray(params, np.float32)
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.size}")
        self._host(self.ctx.lib.argus_cnn_set_weights, p)

    def get_weights(self):
        return self._host(self.ctx.lib.argus_cnn_get_weights)

    def get_grads(self):
        return self._host(self.ctx.lib.argus_cnn_get_grads)

    def forward(self, X, valid, out):
        torch = self.ctx._torch
        self.ctx._bind()
        T = int(valid.shape[0])
        self.ctx._check(self.ctx.lib.argus_cnn_forward(
            self.ctx.h, self.h, _ptr(X, torch.bfloat16), _ptr(valid, torch.uint8), T,
            _ptr(out, torch.float32)))

    def train_step(self, X, valid, target, lr, loss):
        torch = self.ctx._torch
        self.ctx._bind()
        T = int(valid.shape[0])
        self.ctx._check(self.ctx.lib.argus_cnn_train_step(
            self.ctx.h, self.h, _ptr(X, torch.bfloat16), _ptr(valid, torch.uint8),
            _ptr(target, torch.float32), T, float(lr), _ptr(loss, torch.float64)))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.argus_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cnn_param_layout(C_=32, cin=2, nout=31):
    """Slices of the flat parameter vector: per layer w [32][9][c_in] and b [32],
    then the head [nout][32] and its nout biases."""
    out, off = {}, 0
    ch = [cin, C_, C_, C_, C_]
    for l in range(4):
        n = ch[l + 1] * 9 * ch[l]
        out[f"w{l}"] = (slice(off, off + n), (ch[l + 1], 9, ch[l]))
        off += n
        out[f"b{l}"] = (slice(off, off + ch[l + 1]), (ch[l + 1],))
        off += ch[l + 1]
    out["hw"] = (slice(off, off + nout * C_), (nout, C_))
    off += nout * C_
    out["hb"] = (slice(off, off + nout), (nout,))
    off += nout
    return out, off
