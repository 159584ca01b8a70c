// libargus C ABI: context, workspace, argument validation and dispatch.
// The operations themselves are specified in include/argus.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "internal.h"

int argus_fail(argus_ctx *ctx, int code, const char *fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

static bool stream_capturing(argus_ctx *ctx) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(ctx->stream, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

int argus_ws_reserve(argus_ctx *ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return ARGUS_OK;
    if (stream_capturing(ctx))
        return argus_fail(ctx, ARGUS_EBUSY, "workspace of %zu bytes needed during stream capture", bytes);
    if (ctx->ws) {
        // work already queued may still read the old buffer
        ARGUS_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
        ARGUS_HIP_CHECK(ctx, hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    size_t want = bytes + (bytes >> 3);
    if (hipMalloc(&ctx->ws, want) != hipSuccess) {
        ctx->ws = nullptr;
        return argus_fail(ctx, ARGUS_ENOMEM, "workspace allocation of %zu bytes failed", want);
    }
    ctx->ws_bytes = want;
    return ARGUS_OK;
}

static hipEvent_t pool_event(argus_ctx *ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

static void release_times(argus_ctx *ctx) {
    for (auto &t : ctx->times) {
        ctx->ev_pool.push_back(t.b);
        ctx->ev_pool.push_back(t.e);
    }
    ctx->times.clear();
    if (ctx->ev_open) ctx->ev_pool.push_back(ctx->ev_open);
    ctx->ev_open = nullptr;
}

void argus_time_begin(argus_ctx *ctx) {
    if (!ctx->timing) return;
    if (!ctx->ev_open) ctx->ev_open = pool_event(ctx);
    if (ctx->ev_open) (void)hipEventRecord(ctx->ev_open, ctx->stream);
}

// name: a string literal (kept by pointer)
void argus_time_end(argus_ctx *ctx, const char *name) {
    if (!ctx->timing || !ctx->ev_open) return;
    hipEvent_t e = pool_event(ctx);
    if (!e) return;
    (void)hipEventRecord(e, ctx->stream);
    ctx->times.push_back({name, ctx->ev_open, e});
    ctx->ev_open = nullptr;
}

// ---- autotuner cache ---------------------------------------------------------
// One JSON object per line, written by this library in a fixed key order:
//   {"key": "<key>", "choice": <int>, "ms": [<float>, ...]}
// Lines that do not parse are skipped; a later line for a key wins.
static void tune_parse_line(argus_ctx *ctx, const char *line) {
    static const char KK[] = "\"key\": \"", KC[] = "\"choice\": ", KM[] = "\"ms\": [";
    const char *k = strstr(line, KK);
    const char *c = strstr(line, KC);
    const char *m = strstr(line, KM);
    if (!k || !c || !m) return;
    k += sizeof KK - 1;
    c += sizeof KC - 1;
    const char *ke = strchr(k, '"');
    if (!ke) return;
    argus_ctx::Tuned t;
    t.key.assign(k, ke - k);
    char *end = nullptr;
    t.choice = (int)strtol(c, &end, 10);
    if (end == c) return;
    const char *q = m + sizeof KM - 1;
    while (*q && *q != ']') {
        float v = strtof(q, &end);
        if (end == q) return;
        t.ms.push_back(v);
        q = end;
        while (*q == ',' || *q == ' ') ++q;
    }
    if (*q != ']' || t.choice < 0 || t.choice >= (int)t.ms.size()) return;
    for (auto &e : ctx->tuned)
        if (e.key == t.key) { e = t; return; }
    ctx->tuned.push_back(t);
}

static void tune_load(argus_ctx *ctx) {
    if (ctx->tune_path.empty()) return;
    FILE *f = fopen(ctx->tune_path.c_str(), "r");
    if (!f) return;                    // no file yet: it is created on the first store
    char line[4096];
    while (fgets(line, sizeof line, f)) tune_parse_line(ctx, line);
    fclose(f);
}

std::string argus_tune_device_key(argus_ctx *ctx) {
    hipDeviceProp_t prop;
    char buf[384];
    int rt = 0;
    if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) prop.gcnArchName[0] = 0;
    if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = 0;
    snprintf(buf, sizeof buf, "device=%s;hip=%d;cu=%d", prop.gcnArchName, rt, ctx->n_cu);
    return buf;
}

const argus_ctx::Tuned *argus_tune_lookup(const argus_ctx *ctx, const std::string &key) {
    for (const auto &e : ctx->tuned)
        if (e.key == key) return &e;
    return nullptr;
}

void argus_tune_store(argus_ctx *ctx, const std::string &key, int choice, const std::vector<float> &ms) {
    argus_ctx::Tuned t{key, choice, ms};
    bool found = false;
    for (auto &e : ctx->tuned)
        if (e.key == key) { e = t; found = true; }
    if (!found) ctx->tuned.push_back(t);
    if (ctx->tune_path.empty()) return;
    FILE *f = fopen(ctx->tune_path.c_str(), "a");
    if (!f) return;                    // an unwritable cache file only loses persistence
    fprintf(f, "{\"key\": \"%s\", \"choice\": %d, \"ms\": [", key.c_str(), choice);
    for (size_t i = 0; i < ms.size(); ++i) fprintf(f, "%s%.6g", i ? ", " : "", ms[i]);
    fprintf(f, "]}\n");
    fclose(f);
}

extern "C" {

int argus_ctx_set_tune_cache(argus_ctx *ctx, const char *path) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    ctx->tune_path = path ? path : "";
    tune_load(ctx);
    return ARGUS_OK;
}

int argus_ctx_create(int device, argus_ctx **out) {
    if (!out) return ARGUS_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return ARGUS_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return ARGUS_EHIP;
    argus_ctx *c = new argus_ctx();
    c->device = device;
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        c->n_cu = 0;
    if (hipMalloc((void **)&c->tables, sizeof(BasisTables)) != hipSuccess) {
        delete c;
        return ARGUS_ENOMEM;
    }
    if (subtract_scratch_init(c) != ARGUS_OK) {
        (void)hipFree(c->tables);
        delete c;
        return ARGUS_EHIP;
    }
    if (const char *tp = getenv("ARGUS_TUNE_CACHE")) {
        c->tune_path = tp;
        tune_load(c);
    }
    *out = c;
    return ARGUS_OK;
}

void argus_ctx_destroy(argus_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->tables) (void)hipFree(ctx->tables);
    if (ctx->fit_stamps) (void)hipFree(ctx->fit_stamps);
    release_times(ctx);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
}

int argus_ctx_set_stream(argus_ctx *ctx, void *hip_stream) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->err.clear();
    return ARGUS_OK;
}

const char *argus_last_error(const argus_ctx *ctx) { return ctx ? ctx->err.c_str() : "null ctx"; }

int argus_ctx_set_timing(argus_ctx *ctx, int enable) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->timing = enable != 0;
    release_times(ctx);
    return ARGUS_OK;
}

float argus_kernel_time_ms(argus_ctx *ctx, const char *kernel) {
    if (!ctx || !kernel) return -1.f;
    double sum = 0.0;
    int n = 0;
    for (auto &t : ctx->times) {
        if (strcmp(t.name, kernel) != 0) continue;
        float ms = -1.f;
        if (hipEventSynchronize(t.e) != hipSuccess ||
            hipEventElapsedTime(&ms, t.b, t.e) != hipSuccess)
            return -1.f;
        sum += ms;
        ++n;
    }
    return n ? (float)(sum / n) : -1.f;
}

static int check_dims(argus_ctx *ctx, argus_dims d) {
    if (d.width < 1 || d.height < 1 || d.pitch < d.width)
        return argus_fail(ctx, ARGUS_ESHAPE, "bad dims %dx%d pitch %lld", d.width, d.height,
                          (long long)d.pitch);
    if ((int64_t)d.height * d.pitch > ((int64_t)1 << 40))
        return argus_fail(ctx, ARGUS_ESHAPE, "image too large");
    return ARGUS_OK;
}

int argus_calibrate(argus_ctx *ctx, argus_dims dims, const uint16_t *raw, const float *dark,
                    const float *flat, const uint8_t *bpm, float gain, float read_noise,
                    uint16_t sat_adu, float *cal, float *var, uint8_t *mask) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if (!raw || !dark || !flat || !cal || !mask)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_calibrate: null pointer");
    if (!(gain > 0.f) || !(read_noise >= 0.f))
        return argus_fail(ctx, ARGUS_EINVAL, "argus_calibrate: gain must be > 0, read noise >= 0");
    return launch_calibrate(ctx, dims, raw, dark, flat, bpm, gain, read_noise, sat_adu, cal, var,
                            mask);
}

int argus_coadd(argus_ctx *ctx, argus_dims dims, int n_frames, const float *const *cal,
                const float *const *var, const uint8_t *const *mask, float kappa, int max_iter,
                float *ref, float *ref_var, uint8_t *ref_mask, uint8_t *n_used) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if (n_frames < 1 || n_frames > ARGUS_MAX_FRAMES)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_coadd: n_frames %d not in 1..8", n_frames);
    if (!cal || !var || !mask || !ref || !ref_var || !ref_mask)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_coadd: null pointer");
    for (int i = 0; i < n_frames; ++i)
        if (!cal[i] || !var[i] || !mask[i])
            return argus_fail(ctx, ARGUS_EINVAL, "argus_coadd: null frame pointer %d", i);
    if (!(kappa > 0.f) || max_iter < 0 || max_iter > 64)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_coadd: kappa > 0 and 0 <= max_iter <= 64");
    return launch_coadd(ctx, dims, n_frames, cal, var, mask, kappa, max_iter, ref, ref_var,
                        ref_mask, n_used);
}

int argus_calibrate_coadd(argus_ctx *ctx, argus_dims dims, int n_frames,
                          const uint16_t *const *raw, const float *dark, const float *flat,
                          const uint8_t *bpm, float gain, float read_noise, uint16_t sat_adu,
                          float kappa, int max_iter, float *ref, float *ref_var,
                          uint8_t *ref_mask, uint8_t *n_used) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if (n_frames < 1 || n_frames > ARGUS_MAX_FRAMES)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_calibrate_coadd: n_frames %d not in 1..8", n_frames);
    if (!raw || !dark || !flat || !ref || !ref_var || !ref_mask)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_calibrate_coadd: null pointer");
    for (int i = 0; i < n_frames; ++i)
        if (!raw[i]) return argus_fail(ctx, ARGUS_EINVAL, "argus_calibrate_coadd: null frame pointer %d", i);
    if (!(gain > 0.f) || !(read_noise >= 0.f))
        return argus_fail(ctx, ARGUS_EINVAL, "argus_calibrate_coadd: gain must be > 0, read noise >= 0");
    if (!(kappa > 0.f) || max_iter < 0 || max_iter > 64)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_calibrate_coadd: kappa > 0 and 0 <= max_iter <= 64");
    return launch_calibrate_coadd(ctx, dims, n_frames, raw, dark, flat, bpm, gain, read_noise,
                                  sat_adu, kappa, max_iter, ref, ref_var, ref_mask, n_used);
}

static int check_spec(argus_ctx *ctx, const argus_kernel_spec *s) {
    if (!s) return argus_fail(ctx, ARGUS_EINVAL, "null kernel spec");
    if (s->n_gauss < 1 || s->n_gauss > 4)
        return argus_fail(ctx, ARGUS_ESHAPE, "n_gauss %d not in 1..4", s->n_gauss);
    for (int g = 0; g < s->n_gauss; ++g) {
        if (!(s->sigma[g] > 0.0) || s->degree[g] < 0 || s->degree[g] > 6)
            return argus_fail(ctx, ARGUS_ESHAPE, "gaussian %d: sigma > 0 and degree 0..6", g);
    }
    if (argus_nbasis(s) > ARGUS_MAX_NB)
        return argus_fail(ctx, ARGUS_ESHAPE, "%d basis functions > %d", argus_nbasis(s), ARGUS_MAX_NB);
    if (argus_nplanes(s) > ARGUS_MAX_PLANES)
        return argus_fail(ctx, ARGUS_ESHAPE, "too many row-filter planes");
    if (s->half_width < 1 || s->half_width > ARGUS_MAX_H)
        return argus_fail(ctx, ARGUS_ESHAPE, "half_width %d not in 1..15", s->half_width);
    if (s->spatial_degree < 0 || s->spatial_degree > ARGUS_MAX_D || s->bg_degree < 0 ||
        s->bg_degree > s->spatial_degree)
        return argus_fail(ctx, ARGUS_ESHAPE, "spatial_degree 0..2 and 0 <= bg_degree <= spatial_degree");
    if (s->tiles_x < 1 || s->tiles_y < 1 || s->tiles_x > 4096 || s->tiles_y > 4096)
        return argus_fail(ctx, ARGUS_ESHAPE, "tiles must be 1..4096 per axis");
    if (s->mode != ARGUS_FIT_GLOBAL && s->mode != ARGUS_FIT_PER_TILE)
        return argus_fail(ctx, ARGUS_EINVAL, "bad fit mode %d", s->mode);
    if (s->precision != ARGUS_FP32 && s->precision != ARGUS_BF16X3 && s->precision != ARGUS_FP64)
        return argus_fail(ctx, ARGUS_EINVAL, "bad precision %d", s->precision);
    return ARGUS_OK;
}

int argus_kernel_dims(const argus_kernel_spec *spec, int *n_unknowns, int *n_solves) {
    int rc = check_spec(nullptr, spec);
    if (rc) return rc;
    int n = argus_nbasis(spec) * argus_npoly(spec->spatial_degree) + argus_npoly(spec->bg_degree);
    if (n_unknowns) *n_unknowns = n;
    if (n_solves) *n_solves = spec->mode == ARGUS_FIT_GLOBAL ? 1 : spec->tiles_x * spec->tiles_y;
    return ARGUS_OK;
}

int argus_fit_kernel(argus_ctx *ctx, argus_dims dims, const argus_kernel_spec *spec,
                     const float *ref, const float *ref_var, const uint8_t *ref_mask,
                     const float *sci, const float *sci_var, const uint8_t *sci_mask,
                     double *coeffs, double *chi2, int64_t *n_fit, int32_t *status) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if ((rc = check_spec(ctx, spec))) return rc;
    if (!ref || !ref_var || !ref_mask || !sci || !sci_var || !sci_mask || !coeffs || !status)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_fit_kernel: null pointer");
    if (spec->tiles_x > dims.width || spec->tiles_y > dims.height)
        return argus_fail(ctx, ARGUS_ESHAPE, "more tiles than pixels");
    float *stamps = nullptr, *bg = nullptr;
    if (chi2) {
        // the stamp buffer for the residual pass, reserved before any launch
        int n, ns;
        (void)argus_kernel_dims(spec, &n, &ns);
        const int K = 2 * spec->half_width + 1;
        const size_t n_st = (size_t)ns * argus_npoly(spec->spatial_degree) * K * K;
        const size_t n_bg = (size_t)ns * argus_npoly(spec->bg_degree);
        const size_t bytes = ((n_st * 4 + 255) & ~(size_t)255) + n_bg * 4;
        if (bytes > ctx->fit_stamps_bytes) {
            if (stream_capturing(ctx))
                return argus_fail(ctx, ARGUS_EBUSY, "chi2 stamp buffer needed during stream capture");
            if (ctx->fit_stamps) {
                ARGUS_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
                ARGUS_HIP_CHECK(ctx, hipFree(ctx->fit_stamps));
                ctx->fit_stamps = nullptr;
                ctx->fit_stamps_bytes = 0;
            }
            if (hipMalloc(&ctx->fit_stamps, bytes) != hipSuccess) {
                ctx->fit_stamps = nullptr;
                return argus_fail(ctx, ARGUS_ENOMEM, "chi2 stamp buffer of %zu bytes", bytes);
            }
            ctx->fit_stamps_bytes = bytes;
        }
        stamps = (float *)ctx->fit_stamps;
        bg = (float *)((char *)ctx->fit_stamps + ((n_st * 4 + 255) & ~(size_t)255));
    }
    if ((rc = launch_basis_tables(ctx, spec))) return rc;
    rc = launch_fit(ctx, dims, spec, ref, ref_var, ref_mask, sci, sci_var, sci_mask, coeffs,
                    n_fit, status);
    if (rc || !chi2) return rc;
    // second pass over the residuals: D = S - X a at every fit pixel
    if ((rc = launch_expand(ctx, spec, coeffs, stamps, bg))) return rc;
    rc = launch_subtract(ctx, dims, spec, stamps, bg, ref, ref_var, ref_mask, sci, sci_var,
                         sci_mask, nullptr, nullptr, nullptr, chi2, nullptr, nullptr, nullptr);
    if (rc) return rc;
    int n_unk, n_solves;
    (void)argus_kernel_dims(spec, &n_unk, &n_solves);
    return launch_chi2_failed(ctx, chi2, status, n_solves);
}

int argus_expand_kernel(argus_ctx *ctx, const argus_kernel_spec *spec, const double *coeffs,
                        float *stamps, float *bg) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_spec(ctx, spec);
    if (rc) return rc;
    if (!coeffs || !stamps || !bg) return argus_fail(ctx, ARGUS_EINVAL, "argus_expand_kernel: null pointer");
    if ((rc = launch_basis_tables(ctx, spec))) return rc;
    return launch_expand(ctx, spec, coeffs, stamps, bg);
}

int argus_subtract(argus_ctx *ctx, argus_dims dims, const argus_kernel_spec *spec,
                   const float *stamps, const float *bg, const float *ref, const float *ref_var,
                   const uint8_t *ref_mask, const float *sci, const float *sci_var,
                   const uint8_t *sci_mask, float *diff, float *diff_var, uint8_t *diff_mask,
                   double *chi2, int64_t *n_chi2, double *sum_wd, double *sum_w) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if ((rc = check_spec(ctx, spec))) return rc;
    if (!stamps || !bg || !ref || !ref_var || !ref_mask || !sci || !sci_var || !sci_mask ||
        !diff || !diff_var || !diff_mask)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_subtract: null pointer");
    if (spec->tiles_x > dims.width || spec->tiles_y > dims.height)
        return argus_fail(ctx, ARGUS_ESHAPE, "more tiles than pixels");
    return launch_subtract(ctx, dims, spec, stamps, bg, ref, ref_var, ref_mask, sci, sci_var,
                           sci_mask, diff, diff_var, diff_mask, chi2, n_chi2, sum_wd, sum_w);
}

int argus_subtract_noalloc(argus_ctx *ctx, argus_dims dims, const argus_kernel_spec *spec,
                           const float *stamps, const float *bg, const float *ref,
                           const float *ref_var, const uint8_t *ref_mask, const float *sci,
                           const float *sci_var, const uint8_t *sci_mask, float *diff,
                           float *diff_var, uint8_t *diff_mask, double *chi2, int64_t *n_chi2,
                           double *sum_wd, double *sum_w) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if ((rc = check_spec(ctx, spec))) return rc;
    if (!stamps || !bg || !ref || !ref_var || !ref_mask || !sci || !sci_var || !sci_mask ||
        !diff || !diff_var || !diff_mask)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_subtract_noalloc: null pointer");
    if (spec->tiles_x > dims.width || spec->tiles_y > dims.height)
        return argus_fail(ctx, ARGUS_ESHAPE, "more tiles than pixels");
    return launch_subtract(ctx, dims, spec, stamps, bg, ref, ref_var, ref_mask, sci, sci_var,
                           sci_mask, diff, diff_var, diff_mask, chi2, n_chi2, sum_wd, sum_w,
                           true);
}

int argus_detect(argus_ctx *ctx, argus_dims dims, const float *diff, const float *diff_var,
                 const uint8_t *diff_mask, float threshold, const float *psf, int psf_half,
                 float *snr, uint8_t *det_mask, argus_candidate *cands, int32_t capacity,
                 int32_t *n_cands) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if (!diff || !diff_var || !diff_mask || !psf || !det_mask || !n_cands)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_detect: null pointer");
    if (capacity < 0 || (capacity > 0 && !cands))
        return argus_fail(ctx, ARGUS_EINVAL, "argus_detect: capacity < 0 or null candidate list");
    if (psf_half < 0 || psf_half > 15)
        return argus_fail(ctx, ARGUS_ESHAPE, "psf_half %d not in 0..15", psf_half);
    if (!(threshold == threshold))
        return argus_fail(ctx, ARGUS_EINVAL, "threshold is NaN");
    return launch_detect(ctx, dims, diff, diff_var, diff_mask, threshold, psf, psf_half, snr,
                         det_mask, cands, capacity, n_cands);
}

int argus_background(argus_ctx *ctx, argus_dims dims, const float *cal, const uint8_t *mask,
                     int box, float *levels, float *grid, float *map) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if (!cal || !mask || !grid) return argus_fail(ctx, ARGUS_EINVAL, "argus_background: null pointer");
    if (box < 4 || box > 64) return argus_fail(ctx, ARGUS_ESHAPE, "box %d not in 4..64", box);
    return launch_background(ctx, dims, cal, mask, box, levels, grid, map);
}

int argus_detect_sources(argus_ctx *ctx, argus_dims dims, const float *cal, const float *var,
                         const uint8_t *mask, const float *grid, int box, float threshold,
                         const float *psf, int psf_half, float *snr, uint8_t *det_mask,
                         argus_source *sources, int32_t capacity, int32_t *n_sources) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if (!cal || !var || !mask || !grid || !psf || !det_mask || !n_sources)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_detect_sources: null pointer");
    if (capacity < 0 || (capacity > 0 && !sources))
        return argus_fail(ctx, ARGUS_EINVAL, "argus_detect_sources: capacity < 0 or null list");
    if (box < 4 || box > 64) return argus_fail(ctx, ARGUS_ESHAPE, "box %d not in 4..64", box);
    if (psf_half < 0 || psf_half > 15)
        return argus_fail(ctx, ARGUS_ESHAPE, "psf_half %d not in 0..15", psf_half);
    if (!(threshold == threshold)) return argus_fail(ctx, ARGUS_EINVAL, "threshold is NaN");
    return launch_detect_sources(ctx, dims, cal, var, mask, grid, box, threshold, psf, psf_half,
                                 snr, det_mask, sources, capacity, n_sources);
}

int argus_coadd_matched(argus_ctx *ctx, argus_dims dims, int n_frames,
                        const float *const *cal, const float *const *var,
                        const uint8_t *const *mask, const float *const *grids, int box,
                        const float *psf, int psf_half, const float *scales,
                        float *score, float *score_var, float *snr) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if (n_frames < 1 || n_frames > ARGUS_MAX_FRAMES)
        return argus_fail(ctx, ARGUS_EINVAL, "n_frames %d not in 1..%d", n_frames, ARGUS_MAX_FRAMES);
    if (!cal || !var || !mask || !psf || !score || !score_var)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_coadd_matched: null pointer");
    bool any_grid = false;
    for (int j = 0; j < n_frames; ++j) {
        if (!cal[j] || !var[j] || !mask[j])
            return argus_fail(ctx, ARGUS_EINVAL, "argus_coadd_matched: null plane of frame %d", j);
        any_grid |= grids && grids[j];
    }
    if (psf_half < 1 || psf_half > 10)
        return argus_fail(ctx, ARGUS_ESHAPE, "psf_half %d not in 1..10", psf_half);
    if (any_grid && (box < 4 || box > 64))
        return argus_fail(ctx, ARGUS_ESHAPE, "box %d not in 4..64", box);
    return launch_coadd_matched(ctx, dims, n_frames, cal, var, mask, grids, box, psf, psf_half,
                                scales, score, score_var, snr);
}

int argus_healpix_tiles(const argus_wcs *wcs, int width, int height, int nside, int step,
                        int32_t *tiles, int capacity, int *n_tiles) {
    if (!wcs || !n_tiles || (capacity > 0 && !tiles) || capacity < 0) return ARGUS_EINVAL;
    if (width < 1 || height < 1 || nside < 1 || nside > (1 << 20) || step < 1) return ARGUS_EINVAL;
    return healpix_tiles(wcs, width, height, nside, step, tiles, capacity, n_tiles);
}

int argus_resample_healpix(argus_ctx *ctx, argus_dims dims, const float *cal, const float *var,
                           const uint8_t *mask, const argus_wcs *wcs, int nside, int m,
                           const int32_t *tiles, int n_tiles, float *out, float *out_var,
                           uint8_t *out_mask) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if (!cal || !var || !mask || !wcs || !tiles || !out || !out_var || !out_mask)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_resample_healpix: null pointer");
    if (nside < 1 || nside > (1 << 20) || m < 1 || m > 4096 || n_tiles < 1 || n_tiles > 65535)
        return argus_fail(ctx, ARGUS_ESHAPE, "nside %d, m %d or n_tiles %d out of range", nside, m,
                          n_tiles);
    return launch_resample_healpix(ctx, dims, cal, var, mask, wcs, nside, m, tiles, n_tiles, out,
                                   out_var, out_mask);
}

int argus_zogy(argus_ctx *ctx, argus_dims dims, const float *new_img, const uint8_t *new_mask,
               const float *ref, const uint8_t *ref_mask, const int32_t *origins, int n_tiles,
               int L, const float *psf_n, const float *psf_r, int psf_half, double Fn, double Fr,
               double sn, double sr, float *D, float *snr, float *flux, uint8_t *mask,
               double *pd2) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    int rc = check_dims(ctx, dims);
    if (rc) return rc;
    if (!new_img || !new_mask || !ref || !ref_mask || !origins || !psf_n || !psf_r || !D || !snr ||
        !flux || !mask)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_zogy: null pointer");
    if (L < 64 || L > 1024 || (L & (L - 1)) != 0)
        return argus_fail(ctx, ARGUS_ESHAPE, "tile side %d is not a power of two in 64..1024", L);
    if (psf_half < 1 || psf_half > 15 || 4 * psf_half + 2 > L)
        return argus_fail(ctx, ARGUS_ESHAPE, "psf_half %d not in 1..15 or too large for L", psf_half);
    if (n_tiles < 1 || n_tiles > 65535)
        return argus_fail(ctx, ARGUS_ESHAPE, "n_tiles %d not in 1..65535", n_tiles);
    if (!(Fn > 0) || !(Fr > 0) || !(sn >= 0) || !(sr >= 0) || !(sn > 0 || sr > 0) ||
        !isfinite(Fn) || !isfinite(Fr) || !isfinite(sn) || !isfinite(sr))
        return argus_fail(ctx, ARGUS_EINVAL, "argus_zogy: bad zero points or noise sigmas");
    return launch_zogy(ctx, dims, new_img, new_mask, ref, ref_mask, origins, n_tiles, L, psf_n,
                       psf_r, psf_half, Fn, Fr, sn, sr, D, snr, flux, mask, pd2);
}

}  // extern "C"
