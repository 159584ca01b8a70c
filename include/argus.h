/*
 * argus.h - C ABI of libargus: PSF-matched difference imaging on MI355X.
 *
 * The calls follow the per-frame reduction that arXiv:2207.14304 describes
 * for the Argus Array:
 *   - calibration masters (darks, flats, bad-pixel masks, noise maps) and
 *     reference frames live on the GPU for a whole pointing (Compute Nodes
 *     section; first paragraph of Pipeline Implementation);
 *   - every full frame is calibrated: dark subtraction, flat fielding, bad
 *     pixel masking (Image Management section);
 *   - references are coadds of many registered frames (Deep Coaddition in
 *     Sky Segments; Transient Alerts);
 *   - transients come from direct, PSF-matched image subtraction against the
 *     reference (Transient Alerts; Table 2, "direct image subtraction").
 * The paper does not print the subtraction algorithm; the kernel model here
 * is the Gaussian-basis kernel with polynomial spatial variation of Alard &
 * Lupton (1998) and Alard (2000), fit by weighted linear least squares.
 *
 * Conventions shared by every call
 *   - Images are row-major [y][x]; argus_dims.pitch is the row stride in
 *     ELEMENTS (>= width) and applies to every image argument of a call.
 *   - Unless marked "host", every pointer is a device pointer on the ctx's
 *     device.  The caller allocates and owns all inputs and outputs; the
 *     library never frees caller memory.  The library owns only its ctx
 *     workspace, grown on first need (never during stream capture).
 *   - Each call validates its arguments on the host and returns ARGUS_OK or a
 *     negative ARGUS_E* code synchronously; argus_last_error() then describes
 *     the failure.  On success the work is enqueued on the ctx stream and the
 *     call returns WITHOUT synchronising.  Data-dependent failures (a
 *     singular fit, candidate overflow) are reported in device outputs.
 *   - Convolution is true convolution: (R (x) K)(x, y) = sum_{u,v} K(u,v)
 *     R(x-u, y-v) with kernel stamps stored K[v+h][u+h].
 *   - Normalised coordinates xt = (2x-(W-1))/(W-1), yt = (2y-(H-1))/(H-1);
 *     spatial monomials P_m = xt^p yt^q ordered p = 0..D outer, q = 0..D-p.
 */
#ifndef ARGUS_H
#define ARGUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define ARGUS_OK        0
#define ARGUS_EINVAL   (-1)   /* null pointer, bad scalar argument          */
#define ARGUS_ESHAPE   (-2)   /* inconsistent sizes / pitch / spec          */
#define ARGUS_ENOMEM   (-3)   /* workspace allocation failed                */
#define ARGUS_EHIP     (-4)   /* a HIP runtime call failed                  */
#define ARGUS_EBUSY    (-5)   /* would allocate while the stream captures   */
/* per-solve status written by argus_fit_kernel (device int32 array)        */
#define ARGUS_ESINGULAR (-20) /* non-positive diagonal or pivot             */
#define ARGUS_ETOOFEW   (-21) /* fewer fit pixels than unknowns             */

/* ---- mask bits (uint8 masks) ------------------------------------------- */
#define ARGUS_BAD    0x01u  /* bad pixel (bpm, flat <= 0, non-finite master) */
#define ARGUS_SAT    0x02u  /* raw >= saturation                             */
#define ARGUS_EDGE   0x04u  /* within the kernel half-width of the border    */
#define ARGUS_NODATA 0x08u  /* no usable frame in the coadd                  */
#define ARGUS_FOOT   0x10u  /* a flagged reference pixel in the footprint    */
#define ARGUS_DET    0x20u  /* SNR >= threshold                              */
#define ARGUS_CAND   0x40u  /* DET and raster-ordered 8-neighbour maximum    */

/* ---- fit modes and precisions ------------------------------------------ */
#define ARGUS_FIT_GLOBAL   0  /* one solve; tiles only order the partial sums */
#define ARGUS_FIT_PER_TILE 1  /* one independent solve per tile              */
#define ARGUS_FP32   0        /* row moments on FP32 MFMA, FP64 row sums     */
#define ARGUS_BF16X3 1        /* hi/lo-split BF16 MFMA, FP32 accumulation    */
#define ARGUS_FP64   2        /* row moments on FP64 MFMA                    */

typedef struct argus_ctx argus_ctx;

typedef struct {
    int32_t width;
    int32_t height;
    int64_t pitch;            /* row stride in elements, >= width */
} argus_dims;

/* Kernel model: n_gauss Gaussians of width sigma[g] times monomials u^i v^j
 * with i + j <= degree[g] (g outer, then i, then j), sampled on the integer
 * grid of half-width half_width, normalised so that basis 0 has unit sum and
 * every other basis has zero sum and unit L2 norm.  spatial_degree D is the
 * degree of the polynomial in (xt, yt) multiplying every basis; bg_degree is
 * that of the additive background (<= D).  Unknowns:
 *   n = nb * (D+1)(D+2)/2 + (Dbg+1)(Dbg+2)/2,  nb = number of bases (<= 31).
 * Tiles partition the frame at floor(i*W/tiles_x) (and likewise in y). */
typedef struct {
    int32_t n_gauss;          /* 1..4 */
    double  sigma[4];
    int32_t degree[4];
    int32_t half_width;       /* h, 1..15: stamps are (2h+1)^2 */
    int32_t spatial_degree;   /* 0..2 */
    int32_t bg_degree;        /* 0..spatial_degree */
    int32_t tiles_x, tiles_y; /* >= 1 */
    int32_t mode;             /* ARGUS_FIT_GLOBAL or ARGUS_FIT_PER_TILE */
    int32_t precision;        /* ARGUS_FP32, ARGUS_BF16X3 or ARGUS_FP64 */
} argus_kernel_spec;

typedef struct {
    int32_t x, y;
    float snr, flux, flux_err;
} argus_candidate;

/* gnomonic (TAN) world coordinates of a frame: pixel (x, y) has standard
 * coordinates (xi, eta) = cd * (x - crpix1, y - crpix2) in degrees, cd
 * row-major {cd11, cd12, cd21, cd22}, about the direction (ra0, dec0) in
 * degrees (Calabretta & Greisen 2002). */
typedef struct {
    double ra0, dec0;
    double crpix1, crpix2;
    double cd[4];
} argus_wcs;

/* a source of argus_detect_sources: peak pixel, centroid, peak SNR, PSF flux */
typedef struct {
    int32_t x, y;
    float xc, yc, snr, flux, flux_err;
} argus_source;

/* ---- context ------------------------------------------------------------ */
/* Create a context on HIP device `device`; work goes to the null stream until
 * argus_ctx_set_stream.  One context per host thread. */
int  argus_ctx_create(int device, argus_ctx **out);
void argus_ctx_destroy(argus_ctx *ctx);
/* hip_stream is a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream). */
int  argus_ctx_set_stream(argus_ctx *ctx, void *hip_stream);
/* Tuning cache of the autotuner (argus_batch_run's tile-shape search): each
 * search's outcome -- the chosen candidate and every candidate's time -- is
 * kept on the context under a key naming the device (architecture name and
 * compute-unit count), the HIP runtime version, the kernel, its half width,
 * precision and problem-size bucket (log2 of the cutout count and of the
 * summed cutout area); a later search with the same key takes the stored
 * choice without timing.  With a path (or, at context creation, the file
 * named by the ARGUS_TUNE_CACHE environment variable) the entries are read
 * from that file now and every new one is appended to it, one JSON object
 * per line: {"key": "...", "choice": n, "ms": [t0, t1, ...]}; lines that do
 * not parse are skipped and a later line for a key wins.  NULL or "" keeps
 * the cache in memory only.  A file that cannot be opened only loses
 * persistence (no error). */
int  argus_ctx_set_tune_cache(argus_ctx *ctx, const char *path);
/* Message of the most recent synchronous failure on this ctx ("" if none). */
const char *argus_last_error(const argus_ctx *ctx);
/* Per-kernel timing (for measurement only): while enabled, every launch of
 * an internal kernel is bracketed by HIP events on the context stream, with
 * no synchronisation.  argus_kernel_time_ms waits for the recorded launches
 * of the named kernel ("calibrate", "coadd", "calibrate_coadd", "fit_accum",
 * "fit_reduce", "fit_solve", "subtract", "detect_map", "detect_emit",
 * "background", "background_map", "source_map", "source_emit", "coadd_matched",
 * "healpix_resample", "zogy", "batch") and returns
 * their average device time in ms, or -1 if none was recorded.  Enabling or
 * disabling timing discards the records. */
int  argus_ctx_set_timing(argus_ctx *ctx, int enable);
float argus_kernel_time_ms(argus_ctx *ctx, const char *kernel);

/* ---- calibration (Image Management section) ----------------------------
 * Per pixel:  cal  = (raw - dark) / flat
 *             var  = (max(raw - dark, 0)/gain + read_noise^2/gain^2) / flat^2
 *             mask = BAD if bpm != 0, flat <= 0 or flat/dark not finite;
 *                    SAT if raw >= sat_adu.   BAD pixels get cal = var = 0.
 * raw u16, dark/flat f32 (dark includes bias), bpm u8 (nullable = none);
 * outputs cal f32, var f32 (nullable), mask u8.  gain in e-/ADU (> 0),
 * read_noise in e- (Table 1 quotes 1.7 e-).  Streaming; HBM-bound. */
int argus_calibrate(argus_ctx *ctx, argus_dims dims,
                    const uint16_t *raw, const float *dark, const float *flat,
                    const uint8_t *bpm, float gain, float read_noise,
                    uint16_t sat_adu, float *cal, float *var, uint8_t *mask);

/* ---- reference coadd (Deep Coaddition; Transient Alerts) ----------------
 * n_frames (1..8) registered calibrated frames -> clipped mean per pixel.
 * Start with the frames whose mask has neither BAD nor SAT; up to max_iter
 * times: stop if <= 2 remain; c = median of values, s2 = median of variances
 * (even count: mean of the middle two); reject |x - c| > kappa*sqrt(s2);
 * stop if nothing is rejected or fewer than 2 would remain.  ref = mean,
 * ref_var = sum(var)/m^2, n_used = m (nullable); ref_mask NODATA if no frame
 * was usable (ref = ref_var = 0), SAT if any frame is SAT there.
 * cal/var/mask are HOST arrays of n_frames DEVICE pointers.  Decisions are
 * taken in FP64.  Streaming; HBM-bound. */
int argus_coadd(argus_ctx *ctx, argus_dims dims, int n_frames,
                const float *const *cal, const float *const *var,
                const uint8_t *const *mask, float kappa, int max_iter,
                float *ref, float *ref_var, uint8_t *ref_mask, uint8_t *n_used);

/* ---- fused calibration + reference coadd (Image Management; Deep
 * Coaddition) --------------------------------------------------------------
 * The n_frames (1..8) raw frames of one camera, which share dark, flat and
 * bpm, are calibrated exactly as by argus_calibrate and coadded exactly as by
 * argus_coadd (same gain, read_noise, sat_adu, kappa and max_iter rules),
 * without writing the calibrated frames: only raw frames and masters are
 * read and only ref, ref_var, ref_mask and n_used (nullable) are written.
 * Results are bit-identical to argus_calibrate on each frame followed by
 * argus_coadd.  raw is a HOST array of n_frames DEVICE pointers (u16, the
 * dims' pitch).  Errors as for argus_calibrate and argus_coadd.  Streaming;
 * HBM-bound. */
int argus_calibrate_coadd(argus_ctx *ctx, argus_dims dims, int n_frames,
                          const uint16_t *const *raw, const float *dark, const float *flat,
                          const uint8_t *bpm, float gain, float read_noise, uint16_t sat_adu,
                          float kappa, int max_iter, float *ref, float *ref_var,
                          uint8_t *ref_mask, uint8_t *n_used);

/* Number of unknowns per solve and number of solves for a spec (the kernel
 * model of the direct subtraction, Transient Alerts / Table 2): n as given
 * above the argus_kernel_spec type; one solve for ARGUS_FIT_GLOBAL,
 * tiles_x * tiles_y for ARGUS_FIT_PER_TILE.  Either output is nullable;
 * ARGUS_EINVAL or ARGUS_ESHAPE for an invalid spec. */
int argus_kernel_dims(const argus_kernel_spec *spec, int *n_unknowns, int *n_solves);

/* ---- kernel fit (direct subtraction of Transient Alerts / Table 2) ------
 * Fit set: pixels with h <= x <= W-1-h and h <= y <= H-1-h, sci_mask == 0,
 * ref_mask == 0 over the (2h+1)^2 footprint and sci_var + ref_var > 0;
 * weights w = 1/(sci_var + ref_var).  Design row of pixel p: P_m(p) *
 * (ref (x) B_k)(p) at index k*nP + m, then the background block P_m(p).
 * Normal equations are accumulated per tile (FP32 products, FP64 sums),
 * added in FP64 (all tiles for GLOBAL), Jacobi-scaled and Cholesky-solved in
 * FP64 on the GPU.  Outputs (device): coeffs f64 [n_solves][n] (NaN where the
 * solve failed), chi2 f64 [n_solves] (nullable), n_fit i64 [n_solves]
 * (nullable), status i32 [n_solves] (ARGUS_OK, ARGUS_ESINGULAR or
 * ARGUS_ETOOFEW).  chi2 = sum over the fit set of w (S - X a)^2, taken as a
 * second pass over the residuals: the solution is expanded into stamps and
 * the subtraction below is run without writing its images (the residual of
 * a fit pixel is exactly its difference D); NaN where the solve failed; the
 * degrees of freedom are n_fit - n.  Requesting chi2 costs one pass of
 * argus_subtract and a per-context stamp buffer, allocated on first use
 * (ARGUS_EBUSY if that first use is under stream capture). */
int argus_fit_kernel(argus_ctx *ctx, argus_dims dims, const argus_kernel_spec *spec,
                     const float *ref, const float *ref_var, const uint8_t *ref_mask,
                     const float *sci, const float *sci_var, const uint8_t *sci_mask,
                     double *coeffs, double *chi2, int64_t *n_fit, int32_t *status);

/* ---- kernel expansion (the kernel model of the direct subtraction,
 * Transient Alerts / Table 2; Alard 2000's normalised basis) ---------------
 * K_m = sum_k a_{k nP + m} B_k and bg_m = a_{nb nP + m}, evaluated in FP64.
 * stamps f32 [n_solves][nP][2h+1][2h+1], bg f32 [n_solves][nPbg]. */
int argus_expand_kernel(argus_ctx *ctx, const argus_kernel_spec *spec,
                        const double *coeffs, float *stamps, float *bg);

/* ---- PSF-matched convolution and subtraction (direct image subtraction,
 * Transient Alerts section; Table 2) ----------------------------------------
 * Per pixel p, with K_p = sum_m P_m(p) K_m of the solve owning p:
 *   D = S - (sum_{u,v} K_p(u,v) R(x-u, y-v) + sum_m bg_m P_m(p))
 *   V = var_S + sum_{u,v} K_p(u,v)^2 var_R(x-u, y-v)
 * diff_mask = sci_mask | EDGE (within h of the border) | FOOT (any ref_mask
 * bit in the footprint); D = V = 0 where diff_mask != 0.
 * Over each solve's fit set (diff_mask == 0 and var_S + var_R > 0), with
 * w = 1/(var_S + var_R), FP64 sums (each output f64/i64 [n_solves], nullable):
 * chi2 = sum w D^2, n_chi2 = the set's size, sum_wd = sum w D, sum_w = sum w
 * (the last two give the weighted least-squares background correction
 * sum_wd/sum_w for a caller-supplied kernel).  Stamps and bg as written by
 * argus_expand_kernel (any caller kernel works, e.g. a delta). */
int argus_subtract(argus_ctx *ctx, argus_dims dims, const argus_kernel_spec *spec,
                   const float *stamps, const float *bg,
                   const float *ref, const float *ref_var, const uint8_t *ref_mask,
                   const float *sci, const float *sci_var, const uint8_t *sci_mask,
                   float *diff, float *diff_var, uint8_t *diff_mask,
                   double *chi2, int64_t *n_chi2, double *sum_wd, double *sum_w);

/* ---- subtraction without allocation --------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments, outputs and errors as argus_subtract, bit-identical
 * results, but the per-block partial sums of chi2 / n_chi2 / sum_wd / sum_w
 * live in a fixed scratch array of the library (2 MiB per device, held until
 * the process ends) instead of the ctx workspace, and the call performs no
 * hipMalloc, hipFree or other allocation (nor per-kernel timing records).
 * Limit: the frame (or, PER_TILE, the tiles) may need at most 65536 blocks of
 * 128 x 16 output pixels (ceil(w/128) * ceil(h/16) summed over the solves, w
 * and h a solve's region size; a full 9576 x 6388 frame needs 30000);
 * larger inputs return ARGUS_ESHAPE.  Every call on one GPU shares that
 * GPU's scratch: calls that overlap in time on one GPU (other streams, other
 * contexts, other host threads) race and must be ordered by the caller.
 * Nothing needs clearing between calls: every block writes its partials. */
int argus_subtract_noalloc(argus_ctx *ctx, argus_dims dims, const argus_kernel_spec *spec,
                           const float *stamps, const float *bg,
                           const float *ref, const float *ref_var, const uint8_t *ref_mask,
                           const float *sci, const float *sci_var, const uint8_t *sci_mask,
                           float *diff, float *diff_var, uint8_t *diff_mask,
                           double *chi2, int64_t *n_chi2, double *sum_wd, double *sum_w);

/* ---- detection (Transient Alerts: candidates from the subtraction) --------
 * snr = D/sqrt(V) where diff_mask == 0 and V > 0, else 0 (f32, nullable);
 * det_mask = DET where snr >= threshold, | CAND where additionally snr is
 * strictly above every 8-neighbour earlier in raster order and >= every
 * later one (off-image neighbours count as -inf).  Per candidate, with the
 * caller's unit-sum PSF psf [2r+1][2r+1] (r = psf_half, 0..15) over unmasked
 * in-image pixels: Q = sum P^2/V, flux = (sum P D/V)/Q, flux_err = Q^-1/2
 * (FP64 sums).  cands (device, capacity entries) holds the first `capacity`
 * candidates in raster order; *n_cands (device i32) receives the TRUE count,
 * so *n_cands > capacity signals truncation. */
int argus_detect(argus_ctx *ctx, argus_dims dims,
                 const float *diff, const float *diff_var, const uint8_t *diff_mask,
                 float threshold, const float *psf, int psf_half,
                 float *snr, uint8_t *det_mask,
                 argus_candidate *cands, int32_t capacity, int32_t *n_cands);

/* ---- background map (Pipeline Implementation: calibration and source
 * detection on the GPU; Compute Nodes: background and noise maps kept with
 * the calibration frames; Table 2, "median-filtered background map") -------
 * The frame is cut into box x box cells from the origin (box 4..64; the last
 * cell of a row or column spans the remainder).  levels[c] (f32 [gy][gx],
 * gx = ceil(W/box), gy = ceil(H/box), nullable) = the exact median of the
 * cell's calibrated values with mask == 0 (an even count: the mean of the
 * middle pair, rounded once to FP32), NaN where the cell has none.
 * grid[c] (f32 [gy][gx]) = the median of the levels present in the cell's
 * 3 x 3 neighbourhood of cells (0 if none).  map (f32 [H][W] with the dims'
 * pitch, nullable) = the bilinear interpolation of grid between cell centres
 * ((x0 + x1 - 1)/2 of a cell spanning [x0, x1)), held constant beyond the
 * outer centres.  cal f32 and mask u8 as written by argus_calibrate.
 * Errors: ARGUS_EINVAL for null inputs or grid, ARGUS_ESHAPE for box outside
 * 4..64.  With levels null the ctx workspace holds them. */
int argus_background(argus_ctx *ctx, argus_dims dims, const float *cal, const uint8_t *mask,
                     int box, float *levels, float *grid, float *map);

/* ---- full-frame source detection (Pipeline Implementation; Table 2,
 * "source detection") ------------------------------------------------------
 * argus_detect on D = cal - background (grid of argus_background with the
 * same box, evaluated per pixel as its map), V = var and mask = the
 * calibration mask: snr (nullable), det_mask (DET, CAND), and per source, in
 * raster order, the peak pixel, its SNR, the PSF-weighted flux and error, and
 * the centroid (xc, yc) = (x, y) + sum (u, v) max(D, 0) / sum max(D, 0) over
 * the unmasked in-image 3 x 3 neighbourhood (NaN if that sum is 0).
 * sources (device, capacity entries); *n_sources (device i32) receives the
 * true count.  Errors as for argus_detect and argus_background. */
int argus_detect_sources(argus_ctx *ctx, argus_dims dims, const float *cal, const float *var,
                         const uint8_t *mask, const float *grid, int box, float threshold,
                         const float *psf, int psf_half, float *snr, uint8_t *det_mask,
                         argus_source *sources, int32_t capacity, int32_t *n_sources);

/* ---- matched-filter coadd (Deep Coaddition in Sky Segments: a per-image
 * matched filter, the optimal coaddition for point-source detection in
 * background-limited images of Zackay & Ofek 2017) -------------------------
 * For n_frames (1..8) registered images j with variance var_j, mask_j and an
 * optional background grid grid_j (argus_background with the given box;
 * grids or any entry may be null: no background), PSF P_j (psf: device f32
 * [n_frames][2r+1][2r+1], r = psf_half 1..10, unit sum, P[dv+r][du+r] for the
 * offset (du, dv)) and flux zero point F_j (scales: HOST f32 [n_frames], null
 * = all 1), per pixel q with M_j = cal_j - background_j:
 *   score(q)     = sum_j F_j   sum_u P_j(u)   M_j(q+u) / var_j(q+u)
 *   score_var(q) = sum_j F_j^2 sum_u P_j(u)^2 / var_j(q+u)
 * over in-image pixels q+u with mask_j == 0 and var_j > 0; snr (nullable) =
 * score / sqrt(score_var), 0 where score_var == 0.  score_var is the
 * variance of score for independent pixel noise; score / score_var is the
 * PSF flux of a point source at q (in units of F = 1) and score_var^-1/2 its
 * error.  cal/var/mask/grids are HOST arrays of DEVICE pointers; outputs f32
 * with the dims' pitch.  FP32 products, summed in FP32 along a PSF row and in
 * FP64 across rows and images.  Errors: ARGUS_EINVAL (null pointers,
 * n_frames), ARGUS_ESHAPE (psf_half, box). */
int argus_coadd_matched(argus_ctx *ctx, argus_dims dims, int n_frames,
                        const float *const *cal, const float *const *var,
                        const uint8_t *const *mask, const float *const *grids, int box,
                        const float *psf, int psf_half, const float *scales,
                        float *score, float *score_var, float *snr);

/* ---- HEALPix segments (Image Segmentation: every frame reprojected into
 * equal-area NSIDE = 256 sky tiles on the GPU; Table 2, "image segmentation
 * and resampling to HEALPix grid") -----------------------------------------
 * Geometry: the HEALPix projection (Gorski et al. 2005) maps the sphere to
 * a plane where the 12 base pixels are diamonds; face coordinates (a, b) in
 * [0, 1]^2 run from a diamond's south corner to its east (a) and west (b)
 * corners; base pixel f is centred at (pi/4 + f pi/2, pi/4) for f = 0..3,
 * ((f-4) pi/2, 0) for 4..7 and (pi/4 + (f-8) pi/2, -pi/4) for 8..11.  Tile
 * (f, I, J) of NSIDE nside covers a in [I, I+1)/nside, b in [J, J+1)/nside.
 *
 * argus_healpix_tiles (host only): the tiles (f, I, J) that the frame's
 * pixels fall in, sampled every `step` pixels along x and y and along the
 * last row and column, sorted (f, I, J) ascending, into the HOST array tiles
 * [capacity][3]; *n_tiles (host) receives the true count.  ARGUS_EINVAL for
 * null pointers, a singular cd or non-positive sizes.
 *
 * argus_resample_healpix: for each of n_tiles tiles (DEVICE i32 [n][3]) an
 * m x m segment image whose pixel (p, q) (row q) is the HEALPix pixel of
 * NSIDE nside*m at a = (I m + p + 1/2)/(nside m), b = (J m + q + 1/2)/(nside m):
 * the frame is bilinearly interpolated at that direction's frame position
 * (wcs): out = sum w cal, out_var = sum w^2 var over the four neighbours
 * (FP64 weights), out_mask 0; NODATA (out = out_var = 0) where the position
 * is off [0, W-1] x [0, H-1], behind the tangent plane, or a neighbour is
 * masked.  Outputs f32/f32/u8 [n_tiles][m][m].  nside 1..2^20, m 1..4096.
 * FP64 geometry.  Errors: ARGUS_EINVAL (null pointers, singular cd),
 * ARGUS_ESHAPE (sizes). */
int argus_healpix_tiles(const argus_wcs *wcs, int width, int height, int nside, int step,
                        int32_t *tiles, int capacity, int *n_tiles);
int argus_resample_healpix(argus_ctx *ctx, argus_dims dims, const float *cal, const float *var,
                           const uint8_t *mask, const argus_wcs *wcs, int nside, int m,
                           const int32_t *tiles, int n_tiles, float *out, float *out_var,
                           uint8_t *out_mask);

/* ---- ZOGY subtraction (Transient Alerts: the algorithm of Zackay, Ofek &
 * Gal-Yam 2016 for the 30-second cadence and deep coadds; Table 2, "ZOGY
 * image subtraction") -------------------------------------------------------
 * On n_tiles square tiles of side L (a power of two, 64..1024) at origins
 * (DEVICE i32 [n][2]: x0, y0; tiles may overlap or leave the frame) of the
 * background-subtracted new image N and reference R (f32 with masks u8; a
 * masked or off-frame pixel enters both as 0), with unit-sum PSF stamps psf_n,
 * psf_r (DEVICE f32 [2r+1]^2, r = psf_half 1..15, 4r + 2 <= L), flux zero
 * points Fn, Fr > 0 and background noise sigmas sn, sr >= 0 (not both 0),
 * in the Fourier domain of the periodic tile:
 *   den = sqrt(sn^2 Fr^2 |Pr^|^2 + sr^2 Fn^2 |Pn^|^2),
 *   D^ = (Fr Pr^ N^ - Fn Pn^ R^)/den  (0 where den = 0),
 *   F_D = Fn Fr / sqrt(sn^2 Fr^2 + sr^2 Fn^2),  P_D^ = Fr Fn Pr^ Pn^/(F_D den),
 *   S^ = D^ conj(P_D^);
 * outputs per tile pixel (f32/u8 [n][L][L]): D (white, unit variance for
 * white input noise of the given sigmas), snr = S/sqrt(sum P_D^2), flux =
 * S/(F_D sum P_D^2) (the flux of a point source there), mask = EDGE within r
 * of the tile border | FOOT within 2r (Chebyshev) of a masked or off-frame
 * pixel, with D = snr = flux = 0 where flagged.  sum P_D^2 is written to
 * pd2 (DEVICE f64, nullable).  FP64 transforms and arithmetic; workspace
 * grows to about 70 n L^2 bytes.  Errors: ARGUS_EINVAL (null pointers,
 * scalars), ARGUS_ESHAPE (L, r, n). */
int argus_zogy(argus_ctx *ctx, argus_dims dims, const float *new_img, const uint8_t *new_mask,
               const float *ref, const uint8_t *ref_mask, const int32_t *origins, int n_tiles,
               int L, const float *psf_n, const float *psf_r, int psf_half, double Fn, double Fr,
               double sn, double sr, float *D, float *snr, float *flux, uint8_t *mask,
               double *pd2);

/* ---- batched cutouts (per-segment subtraction, Transient Alerts; Table 2) --
 * Many target cutouts from many cameras' frames, each fit with its own
 * spatially constant kernel and differenced, in ONE persistent launch that
 * workgroups drain from a work queue (largest cutouts first), captured in a
 * HIP graph.  Each cutout is treated as a standalone image of side L: its
 * fit set, edges and footprints stay inside the cutout (the same result as
 * argus_fit_kernel / argus_subtract / argus_detect on an L x L copy).
 * Spec: spatial_degree = bg_degree = 0, mode GLOBAL, precision FP32 or
 * FP64 (row moments; FP64 for small, poorly conditioned cutouts),
 * half_width 4..10.  Outputs per cutout c (device):
 *   diff/diff_var (f32), diff_mask/det_mask (u8): L*L values at
 *   out_offset[c], row-major with pitch L (the caller sizes the arena);
 *   coeffs f64 [n][n_unknowns], chi2 f64 [n], n_fit i64 [n],
 *   status i32 [n], n_cands i32 [n] (candidates of det_mask, threshold as
 *   in argus_detect). */
typedef struct {
    int32_t frame;            /* index into the frame table */
    int32_t x0, y0;           /* top-left pixel in the frame */
    int32_t side;             /* L, 2h+2 .. 512 */
    int64_t out_offset;       /* element offset of the cutout in the arena */
} argus_cutout;

typedef struct {              /* one registered, calibrated frame pair (device) */
    const float *ref, *ref_var;
    const uint8_t *ref_mask;
    const float *sci, *sci_var;
    const uint8_t *sci_mask;
    int32_t width, height;
    int64_t pitch;            /* elements, shared by the six planes */
} argus_frame;

typedef struct argus_batch argus_batch;

/* Validate the HOST cutout table against n_frames frames of the given sizes
 * (widths/heights: HOST arrays), order the work, upload it and size the
 * workspace.  Allocates; call outside stream capture. */
int argus_batch_plan(argus_ctx *ctx, const argus_kernel_spec *spec,
                     const argus_cutout *cutouts, int n_cutouts,
                     const int32_t *frame_widths, const int32_t *frame_heights,
                     int n_frames, argus_batch **out);
/* Run the batch on the frames (HOST array of n_frames descriptors).  The
 * first run times every candidate tile shape and workgroup count on these
 * inputs (the autotuner), keeps the fastest, and captures the queue reset
 * and the persistent kernel in a HIP graph; later runs with the same frame
 * and output pointers replay the graph. */
int argus_batch_run(argus_ctx *ctx, argus_batch *batch, const argus_frame *frames,
                    float threshold, float *diff, float *diff_var, uint8_t *diff_mask,
                    uint8_t *det_mask, double *coeffs, double *chi2, int64_t *n_fit,
                    int32_t *status, int32_t *n_cands);
/* Autotuner outcome: chosen candidate index, its time in ms, and the number of
 * candidates tried (any pointer may be null). */
int argus_batch_info(const argus_batch *batch, int *choice, float *ms, int *n_candidates);
/* Every candidate's time in ms, in candidate order (the first `capacity`
 * are written to cand_ms), their number, and whether the choice was taken
 * from the context's tuning cache (then the times are the stored ones).
 * Before the first run the count is 0. */
int argus_batch_tuning(const argus_batch *batch, float *cand_ms, int capacity, int *n_candidates,
                       int *from_cache);
/* Shape of autotuner candidate `index`: subtraction tile height in rows and
 * workgroups per compute unit of the persistent launch.  ARGUS_EINVAL for an
 * index outside the candidate list. */
int argus_batch_candidate(int index, int *tile_rows, int *wg_per_cu);
void argus_batch_destroy(argus_batch *batch);

/* ---- learned kernel surrogate -------------------------------------------
 * The paper has no learned component.  This one predicts, per tile, the
 * coefficients of the kernel model above (the constant-kernel form of the
 * fit in the difference-imaging step) from paired star stamps; the plain
 * least-squares fit stays the fallback and decides by chi^2/dof where the
 * prediction is kept.
 * Network, shared by every stamp pair of a tile: four 3x3 'same'
 * convolutions (zero padding, cross-correlation) 2 -> 32 -> 32 -> 32 -> 32
 * with bias and ReLU, BF16 weights and activations, FP32 accumulation on
 * MFMA; a spatial mean; the mean over the tile's valid stamps; an FP32
 * linear head to the 31 kernel coefficients.  Loss: mean squared error.
 * Parameters (FP32 master, argus_cnn_n_params floats): per layer the weights
 * [32][9][c_in] (tap = 3 (dy+1) + (dx+1)) then the 32 biases, then the head
 * [31][32] and its 31 biases.  Adam (0.9, 0.999, 1e-8) updates the master.
 * Stamps X are bf16 bit patterns [T][64][31*31][2] (reference, science),
 * 4-byte aligned (a pixel's pair is read as one word; ARGUS_EINVAL
 * otherwise), valid u8 [T][64].  All device pointers unless marked HOST; calls enqueue on
 * the context's stream.  The handle owns its buffers (activations for
 * max_tiles tiles) until argus_cnn_destroy; one handle serves one stream. */
typedef struct argus_cnn argus_cnn;
int  argus_cnn_create(argus_ctx *ctx, int max_tiles, argus_cnn **out);
void argus_cnn_destroy(argus_cnn *cnn);
int  argus_cnn_n_params(const argus_cnn *cnn);
/* HOST copies of the FP32 master parameters; setting them resets Adam. */
int  argus_cnn_set_weights(argus_ctx *ctx, argus_cnn *cnn, const float *host_params);
int  argus_cnn_get_weights(argus_ctx *ctx, argus_cnn *cnn, float *host_params);
/* HOST copy of the gradients of the last train step (before its update). */
int  argus_cnn_get_grads(argus_ctx *ctx, argus_cnn *cnn, float *host_grads);
/* out f32 [T][31] (device). */
int  argus_cnn_forward(argus_ctx *ctx, argus_cnn *cnn, const uint16_t *X, const uint8_t *valid,
                       int T, float *out);
/* One forward + backward + Adam step on T tiles; target f32 [T][31];
 * *loss (device f64) receives the mean squared error before the update. */
int  argus_cnn_train_step(argus_ctx *ctx, argus_cnn *cnn, const uint16_t *X,
                          const uint8_t *valid, const float *target, int T, float lr,
                          double *loss);
/* CNN outputs f32 [n_solves][n_basis] -> coefficients f64
 * [n_solves][n_basis + 1] (constant kernel and background, the layout of
 * argus_fit_kernel with spatial_degree = bg_degree = 0) with zero background. */
int  argus_surrogate_coeffs(argus_ctx *ctx, int n_solves, int n_basis, const float *cnn_out,
                            double *coeffs);
/* Acceptance of the surrogate per solve.  From argus_subtract run with the
 * surrogate's kernel and zero background (chi2_0, n_0, sum_wd, sum_w), the
 * weighted least-squares background b = sum_wd/sum_w gives
 * chi2_s = chi2_0 - sum_wd^2/sum_w on n_0 - 1 degrees of freedom.  The tile
 * keeps the surrogate where chi2_s/(n_0 - 1) <= factor * r_p, with r_p the
 * plain fit's chi2/(n - n_basis - 1) (plain_chi2, plain_n) or, when those
 * are null, the caller's ref_chi2_dof.  coeffs_out f64 [n][n_basis + 1]: the
 * surrogate's kernel and b where accepted, else plain_coeffs (NaN when
 * null); chi2_dof f64 [n] = chi2_s/(n_0 - 1); accepted i32 [n] = 1/0. */
int  argus_surrogate_select(argus_ctx *ctx, int n_solves, int n_basis, const double *sur_coeffs,
                            const double *chi2_0, const int64_t *n_0, const double *sum_wd,
                            const double *sum_w, const double *plain_coeffs,
                            const double *plain_chi2, const int64_t *plain_n,
                            double ref_chi2_dof, double factor, double *coeffs_out,
                            double *chi2_dof, int32_t *accepted);
/* Surrogate inputs of a tiled frame pair: per tile (raster order) the
 * positive reference local maxima (strictly above earlier 8-neighbours in
 * raster order, >= later ones) whose (2 half + 1)^2 stamp lies in the frame
 * and whose peak is >= snr_min sigmas above the tile's sky (the FP32 median
 * of its unmasked reference pixels, by radix select) are ranked brightest
 * first (raster order on ties); walking down the
 * ranking, a candidate is kept when its stamp is unmasked in both frames and
 * (peak - border median of its reference stamp) / sqrt(ref_var at the peak)
 * >= snr_min (FP32), until stamps_per_tile are kept.  Each kept pair loses
 * its border medians; both are multiplied by 100 / (the reference stamp's
 * remaining sum).  X bf16 bits [T][stamps_per_tile][(2 half+1)^2][2]
 * (reference, science), valid u8 [T][stamps_per_tile]; unused slots are zero
 * with valid = 0.  The ranking holds the brightest <= 2048 candidates of a
 * tile; *overflow (device i32, caller-cleared) counts tiles whose walk ran
 * out of retained candidates while dimmer ones had been dropped (their
 * selection can then differ from the definition). */
int  argus_extract_stamps(argus_ctx *ctx, argus_dims dims, const float *ref,
                          const float *ref_var, const uint8_t *ref_mask, const float *sci,
                          const uint8_t *sci_mask, int tiles_x, int tiles_y, float snr_min,
                          int stamps_per_tile, int half, uint16_t *X, uint8_t *valid,
                          int32_t *overflow);

#ifdef __cplusplus
}
#endif
#endif /* ARGUS_H */
