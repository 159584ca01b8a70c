// ZOGY subtraction (Zackay, Ofek & Gal-Yam 2016) on square tiles of a frame
// pair, in FP64 on the GPU.
//
// Per tile of side L (a power of two, 64..1024) at origin (x0, y0):
//   N^, R^ = 2-D FFTs of the new and reference tiles (masked or off-frame
//   pixels 0); with the PSF transforms P_n^, P_r^ (stamps centred on the
//   periodic tile's origin) shared by all tiles,
//     den = sqrt(s_n^2 F_r^2 |P_r^|^2 + s_r^2 F_n^2 |P_n^|^2)
//     D^ = (F_r P_r^ N^ - F_n P_n^ R^) / den,  P_D^ = F_r F_n P_r^ P_n^ / (F_D den)
//     S^ = D^ conj(P_D^),  F_D = F_n F_r / sqrt(s_n^2 F_r^2 + s_r^2 F_n^2);
//   D and S by inverse FFTs; SNR = S / sqrt(sum P_D^2) (Parseval over P_D^),
//   flux = S / (F_D sum P_D^2).  Outputs within r of the tile border are
//   EDGE, within 2r of a masked or off-frame pixel FOOT, and 0 there.
//
// 2-D transforms: rows (radix-2 in LDS, one workgroup per row, twiddles from
// a table), a 32 x 32 LDS transpose, rows again; the spectra stay transposed
// ([k_x][k_y]) for the pointwise step and the inverse transform undoes it.
#include <math.h>

#include "internal.h"

namespace {

typedef double2 cplx;

__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void twiddle_kernel(cplx *tw, int L) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= L / 2) return;
    double s, c;
    sincospi(2.0 * k / L, &s, &c);
    tw[k] = make_double2(c, -s);                       // exp(-2 pi i k / L)
}

// One workgroup per row: bit-reversed load, log2(L) radix-2 stages.
template <bool INV>
__global__ __launch_bounds__(256) void fft_rows_kernel(cplx *data, int L, int lg,
                                                       const cplx *tw) {
    extern __shared__ cplx sm[];
    cplx *row = data + (size_t)blockIdx.x * L;
    const int tid = threadIdx.x;
    for (int i = tid; i < L; i += 256) {
        const int j = (int)(__brev((unsigned)i) >> (32 - lg));
        sm[j] = row[i];
    }
    __syncthreads();
    for (int half = 1; half < L; half <<= 1) {
        const int step = L / (2 * half);
        for (int b = tid; b < L / 2; b += 256) {
            const int pos = b % half, i = (b / half) * 2 * half + pos, j = i + half;
            cplx w = tw[pos * step];
            if (INV) w.y = -w.y;
            const cplx u = sm[i], v = cmul(w, sm[j]);
            sm[i] = make_double2(u.x + v.x, u.y + v.y);
            sm[j] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
    for (int i = tid; i < L; i += 256) row[i] = sm[i];
}

// out[p][x][y] = in[p][y][x] for planes of L x L; 32 x 32 tiles through LDS.
__global__ __launch_bounds__(256) void transpose_kernel(const cplx *in, cplx *out, int L) {
    __shared__ cplx t[32][33];
    const int nb = L / 32;
    const int p = blockIdx.x / (nb * nb), b = blockIdx.x % (nb * nb);
    const int bx = (b % nb) * 32, by = (b / nb) * 32;
    const cplx *src = in + (size_t)p * L * L;
    cplx *dst = out + (size_t)p * L * L;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int r = ty; r < 32; r += 8) t[r][tx] = src[(size_t)(by + r) * L + bx + tx];
    __syncthreads();
    for (int r = ty; r < 32; r += 8) dst[(size_t)(bx + r) * L + by + tx] = t[tx][r];
}

struct ZArgs {
    const float *N, *R;
    const uint8_t *mn, *mr;
    const int32_t *org;                // [n][2]: x0, y0
    int64_t pitch;
    int W, H, L, n, r;
};

// tile planes (real part = value, 0 where masked or off the frame) and the
// tile's bad-pixel map
__global__ void zogy_load_kernel(ZArgs a, cplx *pn, cplx *pr, uint8_t *bad) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, t = blockIdx.z;
    if (x >= a.L) return;
    const int X = a.org[2 * t] + x, Y = a.org[2 * t + 1] + y;
    float vn = 0.f, vr = 0.f;
    uint8_t b = 1;
    if (X >= 0 && X < a.W && Y >= 0 && Y < a.H) {
        const int64_t o = (int64_t)Y * a.pitch + X;
        if (a.mn[o] == 0 && a.mr[o] == 0) {
            vn = a.N[o];
            vr = a.R[o];
            b = 0;
        }
    }
    const size_t i = ((size_t)t * a.L + y) * a.L + x;
    pn[i] = make_double2(vn, 0.0);
    pr[i] = make_double2(vr, 0.0);
    bad[i] = b;
}

// the two PSF stamps wrapped onto the periodic tile (centre at the origin)
__global__ void psf_planes_kernel(const float *pn, const float *pr, int r, int L, cplx *out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= L * L) return;
    const int y = i / L, x = i % L;
    const int dv = y <= L / 2 ? y : y - L, du = x <= L / 2 ? x : x - L;
    double a = 0.0, b = 0.0;
    if (dv >= -r && dv <= r && du >= -r && du <= r) {
        a = pn[(dv + r) * (2 * r + 1) + du + r];
        b = pr[(dv + r) * (2 * r + 1) + du + r];
    }
    out[i] = make_double2(a, 0.0);
    out[(size_t)L * L + i] = make_double2(b, 0.0);
}

struct ZCoef {
    double Fn, Fr, sn2, sr2, FD;
};

__device__ __forceinline__ void zogy_at(const ZCoef &c, cplx Pn, cplx Pr, double &den, cplx &PD) {
    const double an = Pn.x * Pn.x + Pn.y * Pn.y, ar = Pr.x * Pr.x + Pr.y * Pr.y;
    den = sqrt(c.sn2 * c.Fr * c.Fr * ar + c.sr2 * c.Fn * c.Fn * an);
    const cplx pp = cmul(Pr, Pn);
    const double s = den > 0.0 ? c.Fr * c.Fn / (c.FD * den) : 0.0;
    PD = make_double2(s * pp.x, s * pp.y);
}

// sum over frequencies of |P_D^|^2 / L^2 (= sum P_D^2), one workgroup, fixed order
__global__ __launch_bounds__(1024) void zogy_pd2_kernel(const cplx *psf, int L, ZCoef c,
                                                        double *pd2) {
    __shared__ double red[16];
    const size_t n = (size_t)L * L;
    double s = 0.0;
    for (size_t i = threadIdx.x; i < n; i += 1024) {
        double den;
        cplx PD;
        zogy_at(c, psf[i], psf[n + i], den, PD);
        s += PD.x * PD.x + PD.y * PD.y;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 16; ++i) t += red[i];
        *pd2 = t / (double)n;
    }
}

// D^ into the N plane, S^ into the R plane
__global__ void zogy_pointwise_kernel(cplx *pn, cplx *pr, const cplx *psf, int L, int n, ZCoef c) {
    const size_t LL = (size_t)L * L;
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= LL * n) return;
    const size_t f = i % LL;
    double den;
    cplx PD;
    const cplx Pn = psf[f], Pr = psf[LL + f];
    zogy_at(c, Pn, Pr, den, PD);
    cplx D = make_double2(0.0, 0.0);
    if (den > 0.0) {
        const cplx a = cmul(Pr, pn[i]), b = cmul(Pn, pr[i]);
        D = make_double2((c.Fr * a.x - c.Fn * b.x) / den, (c.Fr * a.y - c.Fn * b.y) / den);
    }
    pn[i] = D;
    pr[i] = cmul(D, make_double2(PD.x, -PD.y));
}

// separable dilation of the bad map by 2r (rows, then columns)
__global__ void dilate_rows_kernel(const uint8_t *in, uint8_t *out, int L, int rad) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, t = blockIdx.z;
    if (x >= L) return;
    const uint8_t *row = in + ((size_t)t * L + y) * L;
    uint8_t m = 0;
    for (int u = max(x - rad, 0); u <= min(x + rad, L - 1); ++u) m |= row[u];
    out[((size_t)t * L + y) * L + x] = m;
}

struct ZOut {
    float *D, *snr, *flux;
    uint8_t *mask;
    const uint8_t *rowbad;             // bad map dilated along rows
    const double *pd2;
    double FD;
    int L, r, rad;
};

__global__ void zogy_out_kernel(const cplx *pd, const cplx *ps, ZOut o) {
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, t = blockIdx.z;
    const int L = o.L;
    if (x >= L) return;
    const size_t i = ((size_t)t * L + y) * L + x;
    uint8_t m = (x < o.r || x >= L - o.r || y < o.r || y >= L - o.r) ? ARGUS_EDGE : 0;
    uint8_t b = 0;
    for (int v = max(y - o.rad, 0); v <= min(y + o.rad, L - 1); ++v)
        b |= o.rowbad[((size_t)t * L + v) * L + x];
    if (b) m |= ARGUS_FOOT;
    const double inv = 1.0 / ((double)L * L);
    const double pd2 = *o.pd2;
    const double D = pd[i].x * inv, S = ps[i].x * inv;
    o.D[i] = m ? 0.f : (float)D;
    o.snr[i] = m ? 0.f : (float)(S / sqrt(pd2));
    o.flux[i] = m ? 0.f : (float)(S / (o.FD * pd2));
    o.mask[i] = m;
}

}  // namespace

int launch_zogy(argus_ctx *ctx, argus_dims d, const float *N, const uint8_t *mn, const float *R,
                const uint8_t *mr, const int32_t *origins, int n, int L, const float *psf_n,
                const float *psf_r, int r, double Fn, double Fr, double sn, double sr, float *D,
                float *snr, float *flux, uint8_t *mask, double *pd2_out) {
    int lg = 0;
    while ((1 << lg) < L) ++lg;
    const size_t LL = (size_t)L * L;
    // workspace: 2 tile planes (+ a transpose buffer of the same size), 2 PSF
    // planes (+ transpose), twiddles, two bad maps, sum P_D^2
    const size_t b_pl = (size_t)n * LL * sizeof(cplx);
    const size_t b_psf = 2 * LL * sizeof(cplx);
    const size_t b_tw = (size_t)(L / 2) * sizeof(cplx);
    const size_t b_bad = (size_t)n * LL;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t o_pr = al(b_pl), o_t1 = o_pr + al(b_pl), o_t2 = o_t1 + al(b_pl),
                 o_psf = o_t2 + al(b_pl), o_psft = o_psf + al(b_psf), o_tw = o_psft + al(b_psf),
                 o_bad = o_tw + al(b_tw), o_bad2 = o_bad + al(b_bad), o_pd2 = o_bad2 + al(b_bad),
                 total = o_pd2 + 256;
    int rc = argus_ws_reserve(ctx, total);
    if (rc) return rc;
    char *ws = (char *)ctx->ws;
    cplx *pn = (cplx *)ws, *pr = (cplx *)(ws + o_pr), *t1 = (cplx *)(ws + o_t1),
         *t2 = (cplx *)(ws + o_t2), *psf = (cplx *)(ws + o_psf), *psft = (cplx *)(ws + o_psft),
         *tw = (cplx *)(ws + o_tw);
    uint8_t *bad = (uint8_t *)(ws + o_bad), *bad2 = (uint8_t *)(ws + o_bad2);
    double *pd2 = pd2_out ? pd2_out : (double *)(ws + o_pd2);
    hipStream_t st = ctx->stream;
    const size_t lds = (size_t)L * sizeof(cplx);
    auto fft2 = [&](cplx *a, cplx *tmp, int planes, bool inv) -> int {
        // rows, transpose, rows: the result is transposed ([k_x][k_y]) for the
        // forward transform; the inverse of a transposed spectrum ends upright
        if (inv) {
            hipLaunchKernelGGL(fft_rows_kernel<true>, dim3(planes * L), dim3(256), lds, st, a, L, lg, tw);
            hipLaunchKernelGGL(transpose_kernel, dim3(planes * (L / 32) * (L / 32)), dim3(256), 0, st, a, tmp, L);
            hipLaunchKernelGGL(fft_rows_kernel<true>, dim3(planes * L), dim3(256), lds, st, tmp, L, lg, tw);
        } else {
            hipLaunchKernelGGL(fft_rows_kernel<false>, dim3(planes * L), dim3(256), lds, st, a, L, lg, tw);
            hipLaunchKernelGGL(transpose_kernel, dim3(planes * (L / 32) * (L / 32)), dim3(256), 0, st, a, tmp, L);
            hipLaunchKernelGGL(fft_rows_kernel<false>, dim3(planes * L), dim3(256), lds, st, tmp, L, lg, tw);
        }
        ARGUS_HIP_CHECK(ctx, hipGetLastError());
        return ARGUS_OK;
    };
    argus_time_begin(ctx);
    hipLaunchKernelGGL(twiddle_kernel, dim3((L / 2 + 255) / 256), dim3(256), 0, st, tw, L);
    hipLaunchKernelGGL(psf_planes_kernel, dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, st,
                       psf_n, psf_r, r, L, psf);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    if ((rc = fft2(psf, psft, 2, false))) return rc;          // spectra in psft
    ZCoef c;
    c.Fn = Fn; c.Fr = Fr; c.sn2 = sn * sn; c.sr2 = sr * sr;
    c.FD = Fn * Fr / sqrt(c.sn2 * Fr * Fr + c.sr2 * Fn * Fn);
    hipLaunchKernelGGL(zogy_pd2_kernel, dim3(1), dim3(1024), 0, st, (const cplx *)psft, L, c, pd2);
    ZArgs za{N, R, mn, mr, origins, d.pitch, d.width, d.height, L, n, r};
    hipLaunchKernelGGL(zogy_load_kernel, dim3((L + 255) / 256, L, n), dim3(256), 0, st, za, pn, pr, bad);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    // N and R are adjacent in the workspace only if laid out as one array of
    // 2n planes: transform them separately (each n planes)
    if ((rc = fft2(pn, t1, n, false))) return rc;             // N^ (transposed) in t1
    if ((rc = fft2(pr, t2, n, false))) return rc;             // R^ in t2
    hipLaunchKernelGGL(zogy_pointwise_kernel, dim3((unsigned)((LL * n + 255) / 256)), dim3(256), 0,
                       st, t1, t2, (const cplx *)psft, L, n, c);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    if ((rc = fft2(t1, pn, n, true))) return rc;              // D (upright) in pn
    if ((rc = fft2(t2, pr, n, true))) return rc;              // S in pr
    const int rad = 2 * r;
    hipLaunchKernelGGL(dilate_rows_kernel, dim3((L + 255) / 256, L, n), dim3(256), 0, st,
                       (const uint8_t *)bad, bad2, L, rad);
    ZOut o{D, snr, flux, mask, bad2, pd2, c.FD, L, r, rad};
    hipLaunchKernelGGL(zogy_out_kernel, dim3((L + 255) / 256, L, n), dim3(256), 0, st,
                       (const cplx *)pn, (const cplx *)pr, o);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "zogy");
    return ARGUS_OK;
}
