"""FP64 CPU oracle for PSF-matched difference imaging.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (the HIP library and its Python binding) never calls it, and it shares
no code, table or constant generator with that path.

Everything here is plain numpy float64: direct 2-D sums for convolutions,
explicit normal equations with a written-out Cholesky, per-pixel formulas.
Library primitives (a tensordot, a median) serve as single steps only.

Passages followed (the paper is arXiv:2207.14304):

* calibration - Image Management section (dark subtraction, flat fielding,
  bad-pixel masking), Compute Nodes section (per-camera darks, flats, bad-pixel
  masks and noise maps), read noise from Table 1;
* reference coadd from several frames - Deep Coaddition and Transient Alerts
  sections (long-term coadds serve as subtraction references);
* PSF-matched direct subtraction - Transient Alerts section and Table 2
  (direct subtraction per tile); the kernel model is the Gaussian basis with
  polynomial spatial variation of Alard & Lupton (1998, ApJ 503, 325) and
  Alard (2000, A&AS 144, 363), fit by least squares;
* detection - Transient Alerts section (candidates from the subtraction,
  5-sigma peak significance of the injected transient in Fig. 3).

Where the paper is silent the module docstrings state the reading taken.
"""
from .core import (BAD, SAT, EDGE, NODATA, FOOT, DET, CAND,  # noqa: F401
                   KernelSpec, calibrate, coadd, basis, basis_meta, convolve,
                   monomials, norm_coords, tile_bounds, fit_set, design_rows,
                   normal_equations, cholesky, solve, fit_kernel, chi2,
                   expand_kernel, subtract, subtract_at, detect, n_unknowns)
