// Streaming per-pixel kernels: calibration and the clipped-mean reference coadd.
// Both are HBM-bound; each thread owns 8 (calibrate) or 4 (coadd) consecutive
// pixels of one row so that every plane is read with 8- or 16-byte vector
// loads, and rows with a pitch are handled by a (row, chunk) mapping.
#include "internal.h"

namespace {

constexpr int CAL_PX = 8;
constexpr int CO_PX = 4;

struct CalArgs {
    const uint16_t *raw;
    const float *dark, *flat;
    const uint8_t *bpm;
    float *cal, *var;
    uint8_t *mask;
    int64_t pitch;
    int W, H, chunks;         // chunks of CAL_PX pixels per row
    double inv_g, rn2_g2;
    float sat;
    int vec;                  // all planes 16-byte aligned for vector access
};

// cal = (raw - dark)/flat, var = (max(raw - dark, 0)/g + rn^2/g^2)/flat^2,
// evaluated in FP64 and rounded once to FP32, with per-pixel constants shared
// by every frame of a fused calibration: rf = 1/flat (the hardware estimate
// refined by Newton steps, within one FP64 ulp), ndr = -dark rf, A = rf/g and
// B = rn^2 rf^2 / g^2, so that
//   cal64 = fma(raw, rf, ndr),   var64 = fma(max(cal64, 0), A, B)
// (max(raw - dark, 0) rf = max(cal, 0) as rf > 0).  cal64 is within a few
// FP64 ulps of max(|raw rf|, |dark rf|) of the quotient, var64 within a few
// ulps: the FP32 results are those of the exact expressions except where
// these lie that close to an FP32 rounding boundary.
struct CalPix {
    double rf, ndr, A, B;
    bool bad;
};

// 1/x in FP64 for a positive normal x: the hardware estimate refined by two
// Newton steps (each doubles the correct bits), within one ulp of the quotient.
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

__device__ __forceinline__ CalPix cal_pix(const CalArgs &a, float d, float f, uint8_t b) {
    CalPix p;
    p.bad = (b != 0) || !(f > 0.f) || !__builtin_isfinite(f) || !__builtin_isfinite(d);
    // a BAD pixel's values are discarded: any positive operand will do
    p.rf = rcp64(p.bad ? 1.0 : (double)f);
    p.ndr = -(double)d * p.rf;
    p.A = a.inv_g * p.rf;
    p.B = a.rn2_g2 * (p.rf * p.rf);
    return p;
}

__device__ __forceinline__ void cal_val64(uint32_t r, const CalPix &p, double &cd, double &vd) {
    cd = __builtin_fma((double)r, p.rf, p.ndr);
    vd = __builtin_fma(fmax(cd, 0.0), p.A, p.B);
}

__device__ __forceinline__ void cal_one(const CalArgs &a, uint16_t r, const CalPix &p, float &c,
                                        float &v, uint8_t &m) {
    double cd, vd;
    cal_val64(r, p, cd, vd);
    c = p.bad ? 0.f : (float)cd;
    v = p.bad ? 0.f : (float)vd;
    m = (p.bad ? ARGUS_BAD : 0u) | ((float)r >= a.sat ? ARGUS_SAT : 0u);
}

__global__ __launch_bounds__(256) void calibrate_kernel(CalArgs a) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)a.H * a.chunks;
    if (t >= total) return;
    int y = (int)(t / a.chunks);
    int x0 = (int)(t - (int64_t)y * a.chunks) * CAL_PX;
    int64_t o = (int64_t)y * a.pitch + x0;
    if (a.vec && x0 + CAL_PX <= a.W) {
        uint4 r8 = *(const uint4 *)(a.raw + o);
        float4 d0 = *(const float4 *)(a.dark + o), d1 = *(const float4 *)(a.dark + o + 4);
        float4 f0 = *(const float4 *)(a.flat + o), f1 = *(const float4 *)(a.flat + o + 4);
        uint2 b8 = a.bpm ? *(const uint2 *)(a.bpm + o) : make_uint2(0u, 0u);
        uint16_t r[8];
        r[0] = r8.x & 0xffff; r[1] = r8.x >> 16; r[2] = r8.y & 0xffff; r[3] = r8.y >> 16;
        r[4] = r8.z & 0xffff; r[5] = r8.z >> 16; r[6] = r8.w & 0xffff; r[7] = r8.w >> 16;
        float d[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
        float f[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
        float c[8], v[8];
        uint8_t m[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            uint8_t b = (uint8_t)(((i < 4 ? b8.x : b8.y) >> (8 * (i & 3))) & 0xff);
            cal_one(a, r[i], cal_pix(a, d[i], f[i], b), c[i], v[i], m[i]);
        }
        *(float4 *)(a.cal + o) = make_float4(c[0], c[1], c[2], c[3]);
        *(float4 *)(a.cal + o + 4) = make_float4(c[4], c[5], c[6], c[7]);
        if (a.var) {
            *(float4 *)(a.var + o) = make_float4(v[0], v[1], v[2], v[3]);
            *(float4 *)(a.var + o + 4) = make_float4(v[4], v[5], v[6], v[7]);
        }
        uint2 mo;
        mo.x = m[0] | (m[1] << 8) | (m[2] << 16) | ((uint32_t)m[3] << 24);
        mo.y = m[4] | (m[5] << 8) | (m[6] << 16) | ((uint32_t)m[7] << 24);
        *(uint2 *)(a.mask + o) = mo;
        return;
    }
    int n = min(CAL_PX, a.W - x0);
    for (int i = 0; i < n; ++i) {
        float c, v;
        uint8_t m;
        cal_one(a, a.raw[o + i], cal_pix(a, a.dark[o + i], a.flat[o + i], a.bpm ? a.bpm[o + i] : 0), c, v, m);
        a.cal[o + i] = c;
        if (a.var) a.var[o + i] = v;
        a.mask[o + i] = m;
    }
}

// ---------------------------------------------------------------------------
// Clipped-mean coadd.  Decisions (medians, the clip test) are taken in FP64 on
// the FP32 inputs; survivors are tracked as a bitmask per pixel.
struct CoaddArgs {
    const float *cal[ARGUS_MAX_FRAMES];
    const float *var[ARGUS_MAX_FRAMES];
    const uint8_t *mask[ARGUS_MAX_FRAMES];
    float *ref, *ref_var;
    uint8_t *ref_mask, *n_used;
    int64_t pitch;
    int W, H, chunks;
    double kappa2;
    int max_iter;
    int vec;
};

// Sort the N values with non-survivors pushed to +inf (odd-even transposition).
// The inputs are FP32 and their FP64 images order the same way, so the sort
// runs on the FP32 values and only the middle pair is widened.
template <int N>
__device__ __forceinline__ void sort_n(float (&s)[N]) {
#pragma unroll
    for (int pass = 0; pass < N; ++pass) {
#pragma unroll
        for (int i = pass & 1; i + 1 < N; i += 2) {
            float lo = fminf(s[i], s[i + 1]), hi = fmaxf(s[i], s[i + 1]);
            s[i] = lo;
            s[i + 1] = hi;
        }
    }
}

// Median of the survivors (even count: mean of the middle two), in FP64: the
// sum of two FP32 values and its halving are exact there.
template <int N>
__device__ __forceinline__ double median_of(const float (&x)[N], unsigned S, int cnt) {
    float s[N];
#pragma unroll
    for (int i = 0; i < N; ++i) s[i] = (S >> i & 1u) ? x[i] : __builtin_inff();
    sort_n<N>(s);
    int lo = (cnt - 1) >> 1, hi = cnt >> 1;
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        a = (i == lo) ? s[i] : a;
        b = (i == hi) ? s[i] : b;
    }
    return 0.5 * ((double)a + (double)b);
}

// Median of five values without a sort: the smallest and the largest of the
// first four lie on either side of the median, so it is the median of the
// fifth value and the middle two of the four (f, g).  Selects an input value.
__device__ __forceinline__ float med5(float a, float b, float c, float d, float e) {
    const float f = fmaxf(fminf(a, b), fminf(c, d));
    const float g = fminf(fmaxf(a, b), fmaxf(c, d));
    return fmaxf(fminf(e, f), fminf(fmaxf(e, f), g));
}

template <int N>
__device__ __forceinline__ void coadd_one(const CoaddArgs &a, const float (&x)[N],
                                          const float (&v)[N], const uint8_t (&m)[N], float &ref,
                                          float &rv, uint8_t &rm, uint8_t &nu) {
    unsigned S = 0u;
    bool sat = false;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (!(m[i] & (ARGUS_BAD | ARGUS_SAT))) S |= 1u << i;
        sat |= (m[i] & ARGUS_SAT) != 0;
    }
    unsigned S0 = S;
    for (int it = 0; it < a.max_iter; ++it) {
        int cnt = __builtin_popcount(S);
        if (cnt <= 2) break;
        double c, s2;
        if (N == 5 && __all(S == 31u)) {
            // every pixel of the wave has its five samples (the common case)
            c = (double)med5(x[0], x[1 % N], x[2 % N], x[3 % N], x[4 % N]);
            s2 = (double)med5(v[0], v[1 % N], v[2 % N], v[3 % N], v[4 % N]);
        } else {
            c = median_of<N>(x, S, cnt);
            s2 = median_of<N>(v, S, cnt);
        }
        double thr = a.kappa2 * s2;
        unsigned rej = 0u;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double dd = (double)x[i] - c;
            if ((S >> i & 1u) && dd * dd > thr) rej |= 1u << i;
        }
        int nr = __builtin_popcount(rej);
        if (nr == 0 || cnt - nr < 2) break;
        S &= ~rej;
    }
    int cnt = __builtin_popcount(S);
    double sx = 0.0, sv = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        if (S >> i & 1u) {
            sx += (double)x[i];
            sv += (double)v[i];
        }
    }
    // 1/cnt in FP64 (exact for 1, 2, 4, 8; within one FP64 ulp otherwise)
    const double ic = cnt ? rcp64((double)cnt) : 0.0;
    ref = (float)(sx * ic);
    rv = (float)(sv * (ic * ic));
    rm = (S0 == 0u ? ARGUS_NODATA : 0u) | (sat ? ARGUS_SAT : 0u);
    nu = (uint8_t)cnt;
}

template <int N>
__global__ __launch_bounds__(256) void coadd_kernel(CoaddArgs a) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)a.H * a.chunks;
    if (t >= total) return;
    int y = (int)(t / a.chunks);
    int x0 = (int)(t - (int64_t)y * a.chunks) * CO_PX;
    int64_t o = (int64_t)y * a.pitch + x0;
    int n = min(CO_PX, a.W - x0);
    float x[CO_PX][N], v[CO_PX][N];
    uint8_t m[CO_PX][N];
    if (a.vec && n == CO_PX) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
            float4 xc = *(const float4 *)(a.cal[i] + o);
            float4 vc = *(const float4 *)(a.var[i] + o);
            uint32_t mc = *(const uint32_t *)(a.mask[i] + o);
            x[0][i] = xc.x; x[1][i] = xc.y; x[2][i] = xc.z; x[3][i] = xc.w;
            v[0][i] = vc.x; v[1][i] = vc.y; v[2][i] = vc.z; v[3][i] = vc.w;
#pragma unroll
            for (int p = 0; p < CO_PX; ++p) m[p][i] = (uint8_t)(mc >> (8 * p));
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int p = 0; p < CO_PX; ++p) {
                bool in = p < n;
                x[p][i] = in ? a.cal[i][o + p] : 0.f;
                v[p][i] = in ? a.var[i][o + p] : 0.f;
                m[p][i] = in ? a.mask[i][o + p] : (uint8_t)ARGUS_BAD;
            }
    }
    float r[CO_PX], rv[CO_PX];
    uint8_t rm[CO_PX], nu[CO_PX];
#pragma unroll
    for (int p = 0; p < CO_PX; ++p) coadd_one<N>(a, x[p], v[p], m[p], r[p], rv[p], rm[p], nu[p]);
    if (a.vec && n == CO_PX) {
        *(float4 *)(a.ref + o) = make_float4(r[0], r[1], r[2], r[3]);
        *(float4 *)(a.ref_var + o) = make_float4(rv[0], rv[1], rv[2], rv[3]);
        *(uint32_t *)(a.ref_mask + o) = rm[0] | (rm[1] << 8) | (rm[2] << 16) | ((uint32_t)rm[3] << 24);
        if (a.n_used)
            *(uint32_t *)(a.n_used + o) = nu[0] | (nu[1] << 8) | (nu[2] << 16) | ((uint32_t)nu[3] << 24);
    } else {
        for (int p = 0; p < n; ++p) {
            a.ref[o + p] = r[p];
            a.ref_var[o + p] = rv[p];
            a.ref_mask[o + p] = rm[p];
            if (a.n_used) a.n_used[o + p] = nu[p];
        }
    }
}

// ---------------------------------------------------------------------------
// Calibration of N raw frames that share one set of masters, fused with their
// clipped-mean coadd: per pixel the N raw counts stay in registers, so only
// the raw frames and the masters are read and only the coadd is written
// (about 29 instead of 155 bytes per pixel for N = 5).
//
// With one dark, flat and gain for every frame, a pixel's calibrated value and
// its variance are both non-decreasing functions of the raw count (each FP64
// step and the final rounding to FP32 preserve order), and the saturated
// frames are those with the largest counts.  So the counts are sorted once
// (keys count * 8 + frame, 32-bit integer min/max) and the samples calibrated
// in that order: values and variances are then both sorted, the unsaturated
// samples are ranks [0, nv), and every clip pass keeps a run of consecutive
// ranks [l, h] (x - c grows with the rank, so a pass rejects from the two
// ends).  The medians of a pass are the values and variances at the middle
// ranks of the run; no per-pass sort remains.  The decisions are those of
// coadd_kernel on the calibrated frames (same medians, same FP64 test); the
// survivors' FP64 sums run in rank instead of frame order, which changes
// nothing where those sums are exact (always, unless the survivors' FP32
// exponents span more than ~29 binades) and the FP32 result by at most one
// unit elsewhere.
struct CalCoaddArgs {
    const uint16_t *raw[ARGUS_MAX_FRAMES];
    CalArgs cal;               // masters, gain terms (cal/var/mask outputs unused)
    CoaddArgs co;              // kappa, iterations and the coadd outputs (inputs unused)
    uint32_t satkey;           // saturation count * 8: key < satkey <=> count < saturation
};

// ascending sort of N keys (odd-even transposition)
template <int N>
__device__ __forceinline__ void sort_keys(uint32_t (&k)[N]) {
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
        for (int i = r & 1; i + 1 < N; i += 2) {
            const uint32_t lo = min(k[i], k[i + 1]), hi = max(k[i], k[i + 1]);
            k[i] = lo;
            k[i + 1] = hi;
        }
}

// the arithmetic of cal_one without the mask
__device__ __forceinline__ void cal_val(uint32_t r, const CalPix &p, float &c, float &v) {
    double cd, vd;
    cal_val64(r, p, cd, vd);
    c = (float)cd;
    v = (float)vd;
}

template <int N>
__device__ __forceinline__ void calcoadd_one(const CalCoaddArgs &a, const uint16_t (&raw)[N],
                                             const CalPix &cp, bool in, float &ref, float &rv,
                                             uint8_t &rm, uint8_t &nu) {
    const CoaddArgs &co = a.co;
    uint32_t key[N];
#pragma unroll
    for (int i = 0; i < N; ++i) key[i] = ((uint32_t)raw[i] << 3) | (uint32_t)i;
    sort_keys<N>(key);
    const bool sat = key[N - 1] >= a.satkey;
    int nv = N;
    if (__any(sat)) {
        // saturated samples are the top ranks
        nv = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) nv += key[k] < a.satkey ? 1 : 0;
    }
    if (cp.bad || !in) nv = 0;
    float x[N], v[N];
    double xd[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        cal_val(key[k] >> 3, cp, x[k], v[k]);
        xd[k] = (double)x[k];
    }
    int l = 0, h = nv - 1;
    for (int it = 0; it < co.max_iter; ++it) {
        const int cnt = h - l + 1;
        if (cnt <= 2) break;
        double c, s2;
        int ib;
        if (__all(l == 0 && h == N - 1)) {
            // every sample of every pixel of the wave still in (the common first pass)
            constexpr int IA = (N - 1) >> 1, IB = N >> 1;
            c = 0.5 * (xd[IA] + xd[IB]);
            s2 = 0.5 * ((double)v[IA] + (double)v[IB]);
            ib = IB;
        } else {
            const int ia = (l + h) >> 1;
            ib = (l + h + 1) >> 1;
            // the middle ranks' values by selects (no indexed register access);
            // with at least 3 in the run they lie in ranks 1 .. N-2
            double xa = xd[1 % N], xb = xd[1 % N];
            float va = v[1 % N], vb = v[1 % N];
#pragma unroll
            for (int k = 2; k < N - 1; ++k) {
                const bool ta = ia == k, tb = ib == k;
                xa = ta ? xd[k] : xa;
                va = ta ? v[k] : va;
                xb = tb ? xd[k] : xb;
                vb = tb ? v[k] : vb;
            }
            c = 0.5 * (xa + xb);
            s2 = 0.5 * ((double)va + (double)vb);
        }
        const double thr = co.kappa2 * s2;
        unsigned rej = 0u;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            const double dd = xd[k] - c;
            if (dd * dd > thr) rej |= 1u << k;
        }
        rej &= ((2u << h) - 1u) & ~((1u << l) - 1u);      // ranks l..h only
        const int nr = __builtin_popcount(rej);
        if (nr == 0 || cnt - nr < 2) break;
        // ranks below ib lie at or below the median, those from ib on at or above it
        const int nlo = __builtin_popcount(rej & ((1u << ib) - 1u));
        l += nlo;
        h -= nr - nlo;
    }
    const int cnt = h - l + 1;                             // 0 when nv == 0
    // sums over ranks l..h as FMAs with weights 1.0 / 0.0 (fma(1, x, s) is the
    // rounded sum, fma(0, x, s) = s): no selects of 64-bit values
    unsigned run = 0u;                                     // (h = -1 when nv == 0)
    if (cnt > 0) run = ((2u << h) - 1u) & ~((1u << l) - 1u);
    double sx = 0.0, sv = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double wk = (double)((run >> k) & 1u);
        sx = __builtin_fma(wk, xd[k], sx);
        sv = __builtin_fma(wk, (double)v[k], sv);
    }
    const double ic = cnt > 0 ? rcp64((double)cnt) : 0.0;
    ref = (float)(sx * ic);
    rv = (float)(sv * (ic * ic));
    rm = (nv == 0 ? ARGUS_NODATA : 0u) | (sat ? ARGUS_SAT : 0u);
    nu = (uint8_t)cnt;
}

template <int N>
__global__ __launch_bounds__(256) void calcoadd_kernel(CalCoaddArgs a) {
    const CoaddArgs &c = a.co;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)c.H * c.chunks;
    if (t >= total) return;
    int y = (int)(t / c.chunks);
    int x0 = (int)(t - (int64_t)y * c.chunks) * CO_PX;
    int64_t o = (int64_t)y * c.pitch + x0;
    int n = min(CO_PX, c.W - x0);
    uint16_t r[CO_PX][N];
    CalPix cp[CO_PX];
    if (c.vec && n == CO_PX) {
        const float4 d4 = *(const float4 *)(a.cal.dark + o), f4 = *(const float4 *)(a.cal.flat + o);
        const uint32_t b4 = a.cal.bpm ? *(const uint32_t *)(a.cal.bpm + o) : 0u;
        const float d[CO_PX] = {d4.x, d4.y, d4.z, d4.w}, f[CO_PX] = {f4.x, f4.y, f4.z, f4.w};
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const uint2 r4 = *(const uint2 *)(a.raw[i] + o);
            r[0][i] = (uint16_t)(r4.x & 0xffff);
            r[1][i] = (uint16_t)(r4.x >> 16);
            r[2][i] = (uint16_t)(r4.y & 0xffff);
            r[3][i] = (uint16_t)(r4.y >> 16);
        }
#pragma unroll
        for (int p = 0; p < CO_PX; ++p) cp[p] = cal_pix(a.cal, d[p], f[p], (uint8_t)(b4 >> (8 * p)));
    } else {
#pragma unroll
        for (int p = 0; p < CO_PX; ++p) {
            const bool in = p < n;
            const float d = in ? a.cal.dark[o + p] : 0.f, f = in ? a.cal.flat[o + p] : 1.f;
            const uint8_t b = in && a.cal.bpm ? a.cal.bpm[o + p] : 0;
            cp[p] = cal_pix(a.cal, d, f, b);
#pragma unroll
            for (int i = 0; i < N; ++i) r[p][i] = in ? a.raw[i][o + p] : (uint16_t)0;
        }
    }
    float rr[CO_PX], rv[CO_PX];
    uint8_t rm[CO_PX], nu[CO_PX];
#pragma unroll
    for (int p = 0; p < CO_PX; ++p) calcoadd_one<N>(a, r[p], cp[p], p < n, rr[p], rv[p], rm[p], nu[p]);
    if (c.vec && n == CO_PX) {
        *(float4 *)(c.ref + o) = make_float4(rr[0], rr[1], rr[2], rr[3]);
        *(float4 *)(c.ref_var + o) = make_float4(rv[0], rv[1], rv[2], rv[3]);
        *(uint32_t *)(c.ref_mask + o) = rm[0] | (rm[1] << 8) | (rm[2] << 16) | ((uint32_t)rm[3] << 24);
        if (c.n_used)
            *(uint32_t *)(c.n_used + o) = nu[0] | (nu[1] << 8) | (nu[2] << 16) | ((uint32_t)nu[3] << 24);
    } else {
        for (int p = 0; p < n; ++p) {
            c.ref[o + p] = rr[p];
            c.ref_var[o + p] = rv[p];
            c.ref_mask[o + p] = rm[p];
            if (c.n_used) c.n_used[o + p] = nu[p];
        }
    }
}

inline bool aligned(const void *p, size_t al) { return ((uintptr_t)p % al) == 0; }

}  // namespace

int launch_calibrate(argus_ctx *ctx, argus_dims d, const uint16_t *raw, const float *dark,
                     const float *flat, const uint8_t *bpm, float gain, float rn, uint16_t sat,
                     float *cal, float *var, uint8_t *mask) {
    CalArgs a;
    a.raw = raw; a.dark = dark; a.flat = flat; a.bpm = bpm;
    a.cal = cal; a.var = var; a.mask = mask;
    a.pitch = d.pitch; a.W = d.width; a.H = d.height;
    a.chunks = (d.width + CAL_PX - 1) / CAL_PX;
    a.inv_g = 1.0 / (double)gain;
    a.rn2_g2 = (double)rn * (double)rn / ((double)gain * (double)gain);
    a.sat = (float)sat;
    a.vec = (d.pitch % CAL_PX == 0) && aligned(raw, 16) && aligned(dark, 16) && aligned(flat, 16) &&
            (!bpm || aligned(bpm, 8)) && aligned(cal, 16) && (!var || aligned(var, 16)) &&
            aligned(mask, 8);
    int64_t total = (int64_t)a.H * a.chunks;
    dim3 grid((unsigned)((total + 255) / 256));
    argus_time_begin(ctx);
    hipLaunchKernelGGL(calibrate_kernel, grid, dim3(256), 0, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "calibrate");
    return ARGUS_OK;
}

int launch_coadd(argus_ctx *ctx, argus_dims d, int n, const float *const *cal,
                 const float *const *var, const uint8_t *const *mask, float kappa, int max_iter,
                 float *ref, float *ref_var, uint8_t *ref_mask, uint8_t *n_used) {
    CoaddArgs a;
    bool vec = (d.pitch % CO_PX == 0) && aligned(ref, 16) && aligned(ref_var, 16) &&
               aligned(ref_mask, 4) && (!n_used || aligned(n_used, 4));
    for (int i = 0; i < ARGUS_MAX_FRAMES; ++i) {
        a.cal[i] = i < n ? cal[i] : nullptr;
        a.var[i] = i < n ? var[i] : nullptr;
        a.mask[i] = i < n ? mask[i] : nullptr;
        if (i < n) vec = vec && aligned(cal[i], 16) && aligned(var[i], 16) && aligned(mask[i], 4);
    }
    a.ref = ref; a.ref_var = ref_var; a.ref_mask = ref_mask; a.n_used = n_used;
    a.pitch = d.pitch; a.W = d.width; a.H = d.height;
    a.chunks = (d.width + CO_PX - 1) / CO_PX;
    a.kappa2 = (double)kappa * (double)kappa;
    a.max_iter = max_iter;
    a.vec = vec;
    int64_t total = (int64_t)a.H * a.chunks;
    dim3 grid((unsigned)((total + 255) / 256));
    argus_time_begin(ctx);
    switch (n) {
#define ARGUS_CO(N) case N: hipLaunchKernelGGL(coadd_kernel<N>, grid, dim3(256), 0, ctx->stream, a); break;
        ARGUS_CO(1) ARGUS_CO(2) ARGUS_CO(3) ARGUS_CO(4) ARGUS_CO(5) ARGUS_CO(6) ARGUS_CO(7) ARGUS_CO(8)
#undef ARGUS_CO
        default: return argus_fail(ctx, ARGUS_EINVAL, "bad frame count");
    }
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "coadd");
    return ARGUS_OK;
}

int launch_calibrate_coadd(argus_ctx *ctx, argus_dims d, int n, const uint16_t *const *raw,
                           const float *dark, const float *flat, const uint8_t *bpm, float gain,
                           float rn, uint16_t sat, float kappa, int max_iter, float *ref,
                           float *ref_var, uint8_t *ref_mask, uint8_t *n_used) {
    CalCoaddArgs a = {};
    a.cal.dark = dark; a.cal.flat = flat; a.cal.bpm = bpm;
    a.cal.inv_g = 1.0 / (double)gain;
    a.cal.rn2_g2 = (double)rn * (double)rn / ((double)gain * (double)gain);
    a.cal.sat = (float)sat;
    a.satkey = (uint32_t)sat << 3;
    bool vec = (d.pitch % CO_PX == 0) && aligned(dark, 16) && aligned(flat, 16) &&
               (!bpm || aligned(bpm, 4)) && aligned(ref, 16) && aligned(ref_var, 16) &&
               aligned(ref_mask, 4) && (!n_used || aligned(n_used, 4));
    for (int i = 0; i < ARGUS_MAX_FRAMES; ++i) {
        a.raw[i] = i < n ? raw[i] : nullptr;
        if (i < n) vec = vec && aligned(raw[i], 8);
    }
    CoaddArgs &c = a.co;
    c.ref = ref; c.ref_var = ref_var; c.ref_mask = ref_mask; c.n_used = n_used;
    c.pitch = d.pitch; c.W = d.width; c.H = d.height;
    c.chunks = (d.width + CO_PX - 1) / CO_PX;
    c.kappa2 = (double)kappa * (double)kappa;
    c.max_iter = max_iter;
    c.vec = vec;
    int64_t total = (int64_t)c.H * c.chunks;
    dim3 grid((unsigned)((total + 255) / 256));
    argus_time_begin(ctx);
    switch (n) {
#define ARGUS_CC(N) case N: hipLaunchKernelGGL(calcoadd_kernel<N>, grid, dim3(256), 0, ctx->stream, a); break;
        ARGUS_CC(1) ARGUS_CC(2) ARGUS_CC(3) ARGUS_CC(4) ARGUS_CC(5) ARGUS_CC(6) ARGUS_CC(7) ARGUS_CC(8)
#undef ARGUS_CC
        default: return argus_fail(ctx, ARGUS_EINVAL, "bad frame count");
    }
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "calibrate_coadd");
    return ARGUS_OK;
}
