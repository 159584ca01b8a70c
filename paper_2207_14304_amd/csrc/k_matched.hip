// Matched-filter coadd of registered images (the per-image matched filter of
// Zackay & Ofek 2017 that the paper's deep coadds use):
//
//   S(q)   = sum_j F_j   sum_u P_j(u)   M_j(q + u) / V_j(q + u)
//   Var(q) = sum_j F_j^2 sum_u P_j(u)^2            / V_j(q + u)
//
// with M_j = cal_j - bg_j (bg_j the bilinear background of a filtered cell
// grid, or 0), over in-image pixels with mask 0 and V > 0.  One workgroup per
// 128 x 16 output pixels; per image the halo tile of M/V and 1/V is staged in
// LDS (every load of a thread issued before any is used), the image's
// F P and F^2 P^2 taps sit in LDS, and a thread owns 8 consecutive pixels of a
// row with the two windows of a PSF row in registers: 2 FMA per tap, pixel
// and image.  FP32 products summed in FP32 along a PSF row; the row sums are
// added in FP64 (a long FP32 sum over all taps and images lost ~1e-6 of the
// bright stars' scores).
#include "internal.h"
#include "background.h"

namespace {

constexpr int BW = 128, BH = 16, PXT = 8, NTHR = 256;

struct MatchedArgs {
    const float *cal[ARGUS_MAX_FRAMES];
    const float *var[ARGUS_MAX_FRAMES];
    const uint8_t *mask[ARGUS_MAX_FRAMES];
    BgGrid bg[ARGUS_MAX_FRAMES];       // grid == nullptr: no background
    float F[ARGUS_MAX_FRAMES];
    const float *psf;                  // [n][K][K]
    float *S, *Var, *snr;
    int64_t pitch;
    int W, H, n, bx;                   // bx: blocks along x
};

template <int R>
struct MLds {
    static constexpr int K = 2 * R + 1;
    static constexpr int TH = BH + 2 * R;
    static constexpr int TWr = BW + 2 * R;
    static constexpr int TW = (TWr + 3) & ~3;
    static constexpr size_t bytes = (size_t)(2 * TH * TW + 2 * K * K + 8) * 4;
};

template <int R>
__global__ __launch_bounds__(NTHR) void matched_kernel(MatchedArgs a) {
    using L = MLds<R>;
    constexpr int K = L::K, TH = L::TH, TW = L::TW, TWr = L::TWr;
    extern __shared__ __align__(16) float lds[];
    float *At = lds;                   // [TH][TW] M / V
    float *Bt = At + TH * TW;          // [TH][TW] 1 / V
    float *Pt = Bt + TH * TW;          // [K*K][2] F p, F^2 p^2
    const int tid = threadIdx.x;
    const int bx0 = (blockIdx.x % a.bx) * BW, by0 = (blockIdx.x / a.bx) * BH;
    const int64_t P = a.pitch;
    const int ly = tid / (BW / PXT), lx0 = (tid % (BW / PXT)) * PXT;
    // FP32 sums along a PSF row, FP64 across rows and images
    double s[PXT], v[PXT];
#pragma unroll
    for (int i = 0; i < PXT; ++i) { s[i] = 0.0; v[i] = 0.0; }
    for (int j = 0; j < a.n; ++j) {
        __syncthreads();                                  // the previous image's reads are done
        const float *cal = a.cal[j], *var = a.var[j];
        const uint8_t *msk = a.mask[j];
        const BgGrid bg = a.bg[j];
        constexpr int NE = TH * TWr, NH = (NE + NTHR - 1) / NTHR, NB = 8;
        for (int j0 = 0; j0 < NH; j0 += NB) {
            float hc[NB], hv[NB];
            uint8_t hm[NB];
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                const int i = tid + (j0 + e) * NTHR;
                const int ii = i < NE ? i : 0;
                int X = bx0 - R + ii % TWr, Y = by0 - R + ii / TWr;
                X = X < 0 ? 0 : (X >= a.W ? a.W - 1 : X);
                Y = Y < 0 ? 0 : (Y >= a.H ? a.H - 1 : Y);
                const int64_t o = (int64_t)Y * P + X;
                hc[e] = cal[o];
                hv[e] = var[o];
                hm[e] = msk[o];
            }
#pragma unroll
            for (int e = 0; e < NB; ++e) {
                const int i = tid + (j0 + e) * NTHR;
                if (i < NE) {
                    const int cy = i / TWr, cx = i % TWr;
                    const int X = bx0 - R + cx, Y = by0 - R + cy;
                    const bool ok = X >= 0 && X < a.W && Y >= 0 && Y < a.H && hm[e] == 0 &&
                                    hv[e] > 0.f;
                    float m = hc[e];
                    if (bg.grid && ok) m -= bg_at(bg, X, Y);
                    At[cy * TW + cx] = ok ? m / hv[e] : 0.f;
                    Bt[cy * TW + cx] = ok ? 1.f / hv[e] : 0.f;
                }
            }
        }
        const float *pj = a.psf + (size_t)j * K * K;
        const float F = a.F[j];
        for (int t = tid; t < K * K; t += NTHR) {
            const float p = pj[t];
            Pt[2 * t] = F * p;
            Pt[2 * t + 1] = (F * F) * (p * p);
        }
        __syncthreads();
        for (int dv = 0; dv < K; ++dv) {
            // the windows of this PSF row as 16-byte reads (rows are 16-byte
            // aligned; the last read may pass the window by up to three
            // floats, still inside the LDS carve-up)
            constexpr int NW4 = (PXT + 2 * R + 3) / 4;
            const float4 *ra = (const float4 *)(At + (ly + dv) * TW + lx0);
            const float4 *rb = (const float4 *)(Bt + (ly + dv) * TW + lx0);
            float wa[4 * NW4], wb[4 * NW4];
#pragma unroll
            for (int q = 0; q < NW4; ++q) {
                const float4 x4 = ra[q], y4 = rb[q];
                wa[4 * q] = x4.x; wa[4 * q + 1] = x4.y; wa[4 * q + 2] = x4.z; wa[4 * q + 3] = x4.w;
                wb[4 * q] = y4.x; wb[4 * q + 1] = y4.y; wb[4 * q + 2] = y4.z; wb[4 * q + 3] = y4.w;
            }
            float rs[PXT], rv[PXT];
#pragma unroll
            for (int i = 0; i < PXT; ++i) { rs[i] = 0.f; rv[i] = 0.f; }
#pragma unroll
            for (int du = 0; du < K; ++du) {
                const float2 pp = *(const float2 *)(Pt + 2 * (dv * K + du));
#pragma unroll
                for (int i = 0; i < PXT; ++i) {
                    rs[i] += pp.x * wa[i + du];
                    rv[i] += pp.y * wb[i + du];
                }
            }
#pragma unroll
            for (int i = 0; i < PXT; ++i) {
                s[i] += (double)rs[i];
                v[i] += (double)rv[i];
            }
        }
    }
    const int Y = by0 + ly;
    if (Y >= a.H) return;
    const int64_t orow = (int64_t)Y * P;
#pragma unroll
    for (int i = 0; i < PXT; ++i) {
        const int X = bx0 + lx0 + i;
        if (X < a.W) {
            a.S[orow + X] = (float)s[i];
            a.Var[orow + X] = (float)v[i];
            if (a.snr) a.snr[orow + X] = v[i] > 0.0 ? (float)(s[i] / sqrt(v[i])) : 0.f;
        }
    }
}

template <int R>
int matched_launch(argus_ctx *ctx, const MatchedArgs &a, int nblocks) {
    const size_t lds = MLds<R>::bytes;
    ARGUS_HIP_CHECK(ctx, hipFuncSetAttribute((const void *)matched_kernel<R>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(matched_kernel<R>, dim3(nblocks), dim3(NTHR), lds, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

}  // namespace

int launch_coadd_matched(argus_ctx *ctx, argus_dims d, int n, const float *const *cal,
                         const float *const *var, const uint8_t *const *mask,
                         const float *const *grids, int box, const float *psf, int r,
                         const float *scales, float *S, float *Var, float *snr) {
    MatchedArgs a{};
    for (int j = 0; j < n; ++j) {
        a.cal[j] = cal[j];
        a.var[j] = var[j];
        a.mask[j] = mask[j];
        a.F[j] = scales ? scales[j] : 1.f;
        a.bg[j] = (grids && grids[j]) ? make_bg_grid(grids[j], box, d.width, d.height) : BgGrid{};
    }
    a.psf = psf;
    a.S = S; a.Var = Var; a.snr = snr;
    a.pitch = d.pitch; a.W = d.width; a.H = d.height; a.n = n;
    a.bx = (d.width + BW - 1) / BW;
    const int nblocks = a.bx * ((d.height + BH - 1) / BH);
    argus_time_begin(ctx);
    int rc;
    switch (r) {
#define ARGUS_MR(RR) case RR: rc = matched_launch<RR>(ctx, a, nblocks); break;
        ARGUS_MR(1) ARGUS_MR(2) ARGUS_MR(3) ARGUS_MR(4) ARGUS_MR(5) ARGUS_MR(6) ARGUS_MR(7)
        ARGUS_MR(8) ARGUS_MR(9) ARGUS_MR(10)
#undef ARGUS_MR
        default: return argus_fail(ctx, ARGUS_ESHAPE, "psf_half %d not in 1..10", r);
    }
    if (rc) return rc;
    argus_time_end(ctx, "coadd_matched");
    return ARGUS_OK;
}
