// Internal declarations shared by the libargus translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "argus.h"

// Largest supported shapes.
#define ARGUS_MAX_H      15          // kernel half-width
#define ARGUS_MAX_NB     31          // basis functions
#define ARGUS_MAX_PLANES 16          // (gaussian, x-power) row-filter planes
#define ARGUS_MAX_D      2           // spatial degree
#define ARGUS_MAX_FRAMES 8           // coadd inputs
#define ARGUS_MAX_DEVICES 64         // devices with a scratch address table entry
// blocks of 128x16 output pixels whose partial sums fit the fixed scratch of
// argus_subtract_noalloc (4 doubles each: 2 MiB per device)
#define ARGUS_NOALLOC_MAX_BLOCKS 65536

// Device-resident basis tables, laid out in one buffer (floats unless noted).
//   rowf [ARGUS_MAX_PLANES][32]  : exp(-u^2/2s^2) u^i, index u+h
//   colf [32][32]                : alpha_k exp(-v^2/2s^2) v^j, index v+h
//   gam  [32]                    : C'_k = conv_k + gam_k C'_0
//   kpl  [32] (int)              : plane of basis k
//   ipow [ARGUS_MAX_PLANES] (int): x-power i of plane p (filter parity)
//   b2d  [32][31*31] (double)    : normalised 2-D basis B_k[v+h][u+h]
struct BasisTables {
    float rowf[ARGUS_MAX_PLANES][32];
    float colf[32][32];
    float gam[32];
    int32_t kpl[32];
    int32_t nb, nplanes, h, pad;
    int32_t ipow[ARGUS_MAX_PLANES];    // x-power i of each row-filter plane
    double b2d[32][31 * 31];
};

struct argus_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // workspace grown on demand
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // basis tables for the last spec seen
    BasisTables *tables = nullptr;
    bool tables_valid = false;
    argus_kernel_spec tables_spec{};
    // stamps and background of the fit's chi^2 pass (grown on first use)
    void *fit_stamps = nullptr;
    size_t fit_stamps_bytes = 0;
    // optional per-kernel timing: an event pair per timed launch, read back
    // (and averaged per kernel name) only when queried
    bool timing = false;
    struct Timed { const char *name; hipEvent_t b, e; };
    std::vector<Timed> times;
    std::vector<hipEvent_t> ev_pool;
    hipEvent_t ev_open = nullptr;
    int n_cu = 0;                      // compute units of the device
    // autotuner results: key (device, HIP runtime, kernel, shape bucket) ->
    // chosen candidate and every candidate's time; mirrored in a JSON-lines
    // file when tune_path is set
    struct Tuned { std::string key; int choice; std::vector<float> ms; };
    std::vector<Tuned> tuned;
    std::string tune_path;
};

// Loads and stores through a device pointer that addresses global memory, for
// pointers the compiler cannot trace to a kernel argument (loaded from a
// table): the explicit address space gives global rather than flat
// instructions (flat ones also count against the LDS wait counter).
template <class T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ void gst(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}

// Workgroup b of a launch of n runs on XCD b % 8 of the 8 (the dispatcher
// deals workgroups round-robin over the XCDs, each with its own L2).  This
// returns the logical block that b stands for so that every XCD takes one
// contiguous range of logical blocks: neighbouring tiles of a raster order
// (which share halo rows) then share an L2 and run close in time.
constexpr int ARGUS_NXCD = 8;
__device__ __forceinline__ int argus_xcd_block(int b, int n) {
    const int q = n / ARGUS_NXCD, r = n % ARGUS_NXCD;
    const int x = b % ARGUS_NXCD, i = b / ARGUS_NXCD;
    return x * q + (x < r ? x : r) + i;
}

// ---- helpers implemented in argus.hip --------------------------------------
int argus_fail(argus_ctx *ctx, int code, const char *fmt, ...);
int argus_ws_reserve(argus_ctx *ctx, size_t bytes);
// autotuner cache: the key prefix naming this device and HIP runtime, a
// lookup (nullptr if absent) and a store (kept on the ctx, appended to the
// file when one is set)
std::string argus_tune_device_key(argus_ctx *ctx);
const argus_ctx::Tuned *argus_tune_lookup(const argus_ctx *ctx, const std::string &key);
void argus_tune_store(argus_ctx *ctx, const std::string &key, int choice, const std::vector<float> &ms);
void argus_time_begin(argus_ctx *ctx);
void argus_time_end(argus_ctx *ctx, const char *name);

// ---- spec helpers -----------------------------------------------------------
static inline int argus_npoly(int D) { return (D + 1) * (D + 2) / 2; }
static inline int argus_nbasis(const argus_kernel_spec *s) {
    int nb = 0;
    for (int g = 0; g < s->n_gauss; ++g) nb += (s->degree[g] + 1) * (s->degree[g] + 2) / 2;
    return nb;
}
static inline int argus_nplanes(const argus_kernel_spec *s) {
    int np = 0;
    for (int g = 0; g < s->n_gauss; ++g) np += s->degree[g] + 1;
    return np;
}

// ---- kernel launchers (one per translation unit) ----------------------------
int launch_calibrate(argus_ctx *ctx, argus_dims d, const uint16_t *raw, const float *dark,
                     const float *flat, const uint8_t *bpm, float gain, float rn,
                     uint16_t sat, float *cal, float *var, uint8_t *mask);
int launch_calibrate_coadd(argus_ctx *ctx, argus_dims d, int n, const uint16_t *const *raw,
                           const float *dark, const float *flat, const uint8_t *bpm, float gain,
                           float rn, uint16_t sat, float kappa, int max_iter, float *ref,
                           float *ref_var, uint8_t *ref_mask, uint8_t *n_used);
int launch_coadd(argus_ctx *ctx, argus_dims d, int n, const float *const *cal,
                 const float *const *var, const uint8_t *const *mask, float kappa,
                 int max_iter, float *ref, float *ref_var, uint8_t *ref_mask,
                 uint8_t *n_used);
int launch_basis_tables(argus_ctx *ctx, const argus_kernel_spec *spec);
// fill dst (any BasisTables buffer) for spec on the context stream
int launch_basis_tables_to(argus_ctx *ctx, const argus_kernel_spec *spec, BasisTables *dst);
int launch_fit(argus_ctx *ctx, argus_dims d, const argus_kernel_spec *spec,
               const float *ref, const float *ref_var, const uint8_t *ref_mask,
               const float *sci, const float *sci_var, const uint8_t *sci_mask,
               double *coeffs, int64_t *n_fit, int32_t *status);
int launch_expand(argus_ctx *ctx, const argus_kernel_spec *spec, const double *coeffs,
                  float *stamps, float *bg);
// chi2[s] = NaN where status[s] != ARGUS_OK (n solves)
int launch_chi2_failed(argus_ctx *ctx, double *chi2, const int32_t *status, int n);
int launch_subtract(argus_ctx *ctx, argus_dims d, const argus_kernel_spec *spec,
                    const float *stamps, const float *bg, const float *ref,
                    const float *ref_var, const uint8_t *ref_mask, const float *sci,
                    const float *sci_var, const uint8_t *sci_mask, float *diff,
                    float *diff_var, uint8_t *diff_mask, double *chi2, int64_t *n_chi2,
                    double *sum_wd, double *sum_w, bool noalloc = false);
// device address of the fixed scratch of argus_subtract_noalloc for
// ctx->device (which must be current); once per device, at context creation
int subtract_scratch_init(argus_ctx *ctx);
int launch_detect(argus_ctx *ctx, argus_dims d, const float *diff, const float *dvar,
                  const uint8_t *dmask, float thr, const float *psf, int r, float *snr,
                  uint8_t *det, argus_candidate *cands, int32_t cap, int32_t *n_cands);

int launch_background(argus_ctx *ctx, argus_dims d, const float *cal, const uint8_t *mask, int box,
                      float *levels, float *grid, float *map);
int launch_detect_sources(argus_ctx *ctx, argus_dims d, const float *cal, const float *var,
                          const uint8_t *mask, const float *grid, int box, float thr,
                          const float *psf, int r, float *snr, uint8_t *det, argus_source *srcs,
                          int32_t cap, int32_t *n_srcs);

int launch_coadd_matched(argus_ctx *ctx, argus_dims d, int n, const float *const *cal,
                         const float *const *var, const uint8_t *const *mask,
                         const float *const *grids, int box, const float *psf, int r,
                         const float *scales, float *S, float *Var, float *snr);

int launch_resample_healpix(argus_ctx *ctx, argus_dims d, const float *cal, const float *var,
                            const uint8_t *mask, const argus_wcs *wcs, int nside, int m,
                            const int32_t *tiles, int n_tiles, float *out, float *out_var,
                            uint8_t *out_mask);
int healpix_tiles(const argus_wcs *wcs, int W, int H, int nside, int step, int32_t *tiles,
                  int capacity, int *n_tiles);

int launch_zogy(argus_ctx *ctx, argus_dims d, const float *N, const uint8_t *mn, const float *R,
                const uint8_t *mr, const int32_t *origins, int n, int L, const float *psf_n,
                const float *psf_r, int r, double Fn, double Fr, double sn, double sr, float *D,
                float *snr, float *flux, uint8_t *mask, double *pd2_out);

#define ARGUS_HIP_CHECK(ctx, call)                                                 \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return argus_fail((ctx), ARGUS_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)
