// Batched cutouts: each cutout of each camera's frame pair gets its own
// spatially constant kernel fit, convolution, difference and detection map,
// all in ONE persistent launch.  Workgroups pull cutouts from a work queue in
// descending size order (longest-processing-time first), so uneven cutouts
// (64..512 px) balance across the chip; the queue reset and the persistent
// kernel are captured in a HIP graph.  The subtraction tile height and the
// number of workgroups per CU are chosen by timing every candidate on the
// first run (autotuner).
//
// A cutout is a standalone image of side L: the fit uses the same fused
// convolution + MFMA moment code as argus_fit_kernel over its interior,
// followed by an in-LDS FP64 Cholesky of the (nb+1)-unknown system; edges and
// footprints stay inside the cutout.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fit_accum.h"

using argus_fit::FitArgs;
using argus_fit::FitLds;
using argus_fit::NTHR;

struct argus_batch {
    int n = 0, n_frames = 0, n_unk = 0, h = 0, nb = 0, nplanes = 0;
    argus_kernel_spec spec{};
    int8_t plist[4][4];
    void *dev = nullptr;            // device: cutouts, order, frames, queue, basis tables
    BasisTables *d_tables = nullptr;  // the batch's own copy: the context's tables
                                      // change with every other spec used on it
    argus_cutout *d_cuts = nullptr;
    int32_t *d_order = nullptr;
    argus_frame *d_frames = nullptr;
    int32_t *d_queue = nullptr;
    std::vector<int32_t> widths, heights;
    hipStream_t stream = nullptr;   // private stream for the captured graph
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // inputs baked into the captured graph
    std::vector<argus_frame> frames;
    const void *outs[9] = {};
    float thr = 0.f;
    int choice = -1, n_cand = 0;
    float tuned_ms = -1.f;
    std::vector<float> cand_ms;     // every candidate's time (ms), candidate order
    int from_cache = 0;             // the choice came from the context's tuning cache
    int64_t area = 0;               // sum of cutout areas (size bucket of the tuning key)
};

namespace {

constexpr int BW = 128, PXT = 4, DROWS = 4;

struct BatchArgs {
    const argus_frame *frames;
    const argus_cutout *cuts;
    const int32_t *order;
    int32_t *queue;
    const BasisTables *tab;
    int n, nb, nplanes, n_unk;
    int8_t plist[4][4];
    float thr;
    float *diff, *dvar;
    uint8_t *dmask, *det;
    double *coeffs, *chi2;
    int64_t *n_fit;
    int32_t *status, *n_cands;
};

template <int HH, int TILE>
struct BatchLds {
    static constexpr int K = 2 * HH + 1;
    static constexpr int TH = TILE + 2 * HH, TWr = BW + 2 * HH;
    static constexpr int TW = (TWr + 3) & ~3, MW = (TWr + 15) & ~15;
    __host__ __device__ static size_t phase_bytes(int nplanes) {
        size_t fit = FitLds<0, HH>::bytes(nplanes);
        size_t sub = (size_t)2 * TH * TW * 4 + (size_t)TH * MW + (size_t)TH * BW;
        size_t det = (size_t)(DROWS + 2) * (512 + 4) * 4;
        size_t m = fit > sub ? fit : sub;
        m = m > det ? m : det;
        return (m + 255) & ~(size_t)255;
    }
    // after the phase area: moments (801 doubles), solve (n(n+1)/2 + 2n), stamps
    __host__ __device__ static size_t bytes(int nplanes) {
        return phase_bytes(nplanes) + 801 * 8 + (33 * 34 / 2 + 2 * 33 + 8) * 8 + 2 * K * K * 4 + 256;
    }
};

// ---- solve of the (nb+1)-unknown system by wave 0 in LDS --------------------
// Orders this wave's LDS writes before its later reads by other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// G: moments [3][16][16] (blocks (0,0), (0,1), (1,1)), R: rhs [32], cnt.
// Returns the status; the coefficients are left in x[0..n).
__device__ int solve_small(const double *G, const double *R, double cnt, int n, double *L,
                           double *x, double *d, int lane) {
    if (cnt < (double)n) return ARGUS_ETOOFEW;
    // packed lower triangle of the Jacobi-scaled matrix
    for (int r = lane; r < n; r += 64) {
        double dg = G[(r < 16 ? 0 : 512) + (r & 15) * 16 + (r & 15)];
        d[r] = dg > 0.0 ? 1.0 / sqrt(dg) : 0.0;
    }
    wave_sync();
    int bad = 0;
    for (int r = lane; r < n; r += 64) bad |= !(d[r] > 0.0);
    if (__any(bad)) return ARGUS_ESINGULAR;
    for (int r = lane; r < n; r += 64) {
        for (int c = 0; c <= r; ++c) {
            int k = c, l = r;                  // k <= l
            double g;
            if (l < 16) g = G[k * 16 + l];
            else if (k < 16) g = G[256 + k * 16 + (l - 16)];
            else g = G[512 + (k - 16) * 16 + (l - 16)];
            L[r * (r + 1) / 2 + c] = g * d[r] * d[c];
        }
        x[r] = R[r] * d[r];
    }
    wave_sync();
    double mx = 0.0;
    for (int r = lane; r < n; r += 64) mx = fmax(mx, L[r * (r + 1) / 2 + r]);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    const double tol = (double)n * 0x1p-52 * mx;
    for (int j = 0; j < n; ++j) {
        const double piv = L[j * (j + 1) / 2 + j];
        if (!(piv > tol)) return ARGUS_ESINGULAR;
        const double ljj = sqrt(piv);
        wave_sync();
        for (int i = j + 1 + lane; i < n; i += 64) L[i * (i + 1) / 2 + j] /= ljj;
        if (lane == 0) L[j * (j + 1) / 2 + j] = ljj;
        wave_sync();
        for (int i = j + 1 + lane; i < n; i += 64) {
            const double lij = L[i * (i + 1) / 2 + j];
            for (int c = j + 1; c <= i; ++c) L[i * (i + 1) / 2 + c] -= lij * L[c * (c + 1) / 2 + j];
        }
        wave_sync();
    }
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = lane; k < i; k += 64) s += L[i * (i + 1) / 2 + k] * x[k];
        s = wave_sum(s);
        const double v = (x[i] - s) / L[i * (i + 1) / 2 + i];
        wave_sync();
        x[i] = v;
        wave_sync();
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = 0.0;
        for (int k = i + 1 + lane; k < n; k += 64) s += L[k * (k + 1) / 2 + i] * x[k];
        s = wave_sum(s);
        const double v = (x[i] - s) / L[i * (i + 1) / 2 + i];
        wave_sync();
        x[i] = v;
        wave_sync();
    }
    for (int i = lane; i < n; i += 64) x[i] *= d[i];
    wave_sync();
    return ARGUS_OK;
}

template <int HH, int TILE, int PREC>
__device__ void process_cutout(const BatchArgs &a, int c, float *lds) {
    using BL = BatchLds<HH, TILE>;
    constexpr int K = BL::K, TH = BL::TH, TW = BL::TW, MW = BL::MW;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const argus_cutout cu = a.cuts[c];
    // (the frame planes come from a table: loads through them use gld so that
    // they are global, not flat, accesses)
    const argus_frame fr = a.frames[cu.frame];
    const int L = cu.side;
    const int64_t P = fr.pitch;
    const int64_t org = (int64_t)cu.y0 * P + cu.x0;

    char *base = (char *)lds;
    const size_t ph = BL::phase_bytes(a.nplanes);
    double *part = (double *)(base + ph);                      // 801 doubles
    double *Lt = part + 801;                                   // packed factor
    double *xs = Lt + 33 * 34 / 2;                             // solution [33]
    double *dj = xs + 33;                                      // Jacobi scale [33]
    __shared__ int s_status;
    float *Kst = (float *)(dj + 41);                           // stamp, then its square
    float *K2 = Kst + K * K;

    // ---- fit over the cutout interior (same code as argus_fit_kernel) ----
    FitArgs fa;
    fa.ref = fr.ref + org; fa.rvar = fr.ref_var + org; fa.sci = fr.sci + org;
    fa.svar = fr.sci_var + org; fa.rmask = fr.ref_mask + org; fa.smask = fr.sci_mask + org;
    fa.tab = a.tab;
    fa.partials = nullptr;
    fa.pitch = P;
    fa.W = L; fa.H = L; fa.h = HH; fa.nb = a.nb; fa.nplanes = a.nplanes;
    fa.RX = fa.RY = 1; fa.spt = 1; fa.rchunks = 1; fa.stride = 801;
    fa.sx = 0.0; fa.sy = 0.0;
    for (int w = 0; w < 4; ++w)
        for (int j = 0; j < 4; ++j) fa.plist[w][j] = a.plist[w][j];
    {
        FitLds<0, HH> Lf(lds, a.nplanes);
        for (int i = tid; i < 2 * argus_fit::SW * argus_fit::CST; i += NTHR) {
            int k = i % argus_fit::CST;
            if (k >= a.nb && i < argus_fit::SW * argus_fit::CST)
                Lf.cvec[i] = (k == a.nb) ? 1.f : 0.f;
        }
    }
    __syncthreads();
    switch (wave) {
        case 0: argus_fit::fit_wave<0, HH, 0, PREC>(fa, lds, HH, L - HH, HH, L - HH, true, part); break;
        case 1: argus_fit::fit_wave<0, HH, 1, PREC>(fa, lds, HH, L - HH, HH, L - HH, true, part); break;
        case 2: argus_fit::fit_wave<0, HH, 2, PREC>(fa, lds, HH, L - HH, HH, L - HH, true, part); break;
        default: argus_fit::fit_wave<0, HH, 3, PREC>(fa, lds, HH, L - HH, HH, L - HH, true, part); break;
    }
    __syncthreads();
    // ---- solve, expand the stamp ----
    const int n = a.n_unk;
    if (wave == 0) {
        const int st = solve_small(part, part + 768, part[800], n, Lt, xs, dj, lane);
        if (lane == 0) s_status = st;
        double *co = a.coeffs + (size_t)c * n;
        for (int i = lane; i < n; i += 64) co[i] = st == ARGUS_OK ? xs[i] : __builtin_nan("");
        if (lane == 0) {
            a.status[c] = st;
            a.n_fit[c] = (int64_t)part[800];
        }
    }
    __syncthreads();
    const bool ok = s_status == ARGUS_OK;
    for (int t = tid; t < K * K; t += NTHR) {
        double acc = 0.0;
        for (int k = 0; k < a.nb; ++k) acc += xs[k] * a.tab->b2d[k][t];
        const float kf = ok ? (float)acc : __builtin_nanf("");
        Kst[t] = kf;
        K2[t] = kf * kf;
    }
    const float bg = ok ? (float)xs[a.nb] : __builtin_nanf("");
    __syncthreads();

    // ---- convolve, subtract, variance, chi^2 over 128 x TILE tiles ----
    float *Rt = lds, *Vt = Rt + TH * TW;
    uint8_t *Mt = (uint8_t *)(Vt + TH * TW), *Mr = Mt + TH * MW;
    double c2 = 0.0, cnt = 0.0;
    float *dout = a.diff + cu.out_offset, *vout = a.dvar + cu.out_offset;
    uint8_t *mout = a.dmask + cu.out_offset;
    for (int ty0 = 0; ty0 < L; ty0 += TILE) {
        for (int tx0 = 0; tx0 < L; tx0 += BW) {
            // halo: 8 elements per thread in flight at once (clamped
            // addresses, out-of-cutout zeros applied at the store)
            constexpr int NH = (TH * BL::TWr + NTHR - 1) / NTHR, NB8 = 8;
            for (int j0 = 0; j0 < NH; j0 += NB8) {
                float hr[NB8], hv[NB8];
                uint8_t hm[NB8];
#pragma unroll
                for (int j = 0; j < NB8; ++j) {
                    const int i = tid + (j0 + j) * NTHR;
                    const int ii = i < TH * BL::TWr ? i : 0;
                    const int cy = ii / BL::TWr, cx = ii % BL::TWr;
                    int X = tx0 - HH + cx, Y = ty0 - HH + cy;
                    X = X < 0 ? 0 : (X >= L ? L - 1 : X);
                    Y = Y < 0 ? 0 : (Y >= L ? L - 1 : Y);
                    const int64_t o = org + (int64_t)Y * P + X;
                    hr[j] = gld(fr.ref + o);
                    hv[j] = gld(fr.ref_var + o);
                    hm[j] = gld(fr.ref_mask + o);
                }
#pragma unroll
                for (int j = 0; j < NB8; ++j) {
                    const int i = tid + (j0 + j) * NTHR;
                    if (i < TH * BL::TWr) {
                        const int cy = i / BL::TWr, cx = i % BL::TWr;
                        const int X = tx0 - HH + cx, Y = ty0 - HH + cy;
                        const bool in = X >= 0 && X < L && Y >= 0 && Y < L;
                        Rt[cy * TW + cx] = in ? hr[j] : 0.f;
                        Vt[cy * TW + cx] = in ? hv[j] : 0.f;
                        Mt[cy * MW + cx] = (in && hm[j] != 0) ? 1 : 0;
                    }
                }
            }
            __syncthreads();
            for (int i = tid; i < TH * (BW / PXT); i += NTHR) {
                int cy = i / (BW / PXT), lx0 = (i % (BW / PXT)) * PXT;
                uint8_t m[PXT];
#pragma unroll
                for (int px = 0; px < PXT; ++px) m[px] = 0;
#pragma unroll
                for (int j = 0; j < PXT + 2 * HH; ++j) {
                    uint8_t v = Mt[cy * MW + lx0 + j];
#pragma unroll
                    for (int px = 0; px < PXT; ++px)
                        if (j >= px && j <= px + 2 * HH) m[px] |= v;
                }
#pragma unroll
                for (int px = 0; px < PXT; ++px) Mr[cy * BW + lx0 + px] = m[px];
            }
            __syncthreads();
            for (int item = tid; item < TILE * (BW / PXT); item += NTHR) {
                const int ly = item / (BW / PXT), lx0 = (item % (BW / PXT)) * PXT;
                const int Y = ty0 + ly;
                if (Y >= L || tx0 + lx0 >= L) continue;
                float m[PXT], v[PXT];
#pragma unroll
                for (int i = 0; i < PXT; ++i) { m[i] = 0.f; v[i] = 0.f; }
                for (int vv = 0; vv < K; ++vv) {
                    const float *rr = Rt + (ly + 2 * HH - vv) * TW + lx0;
                    const float *qq = Vt + (ly + 2 * HH - vv) * TW + lx0;
                    float r[PXT + 2 * HH], q[PXT + 2 * HH];
#pragma unroll
                    for (int j = 0; j < PXT + 2 * HH; ++j) { r[j] = rr[j]; q[j] = qq[j]; }
#pragma unroll
                    for (int uu = 0; uu < K; ++uu) {
                        const float k = Kst[vv * K + uu], k2 = K2[vv * K + uu];
#pragma unroll
                        for (int i = 0; i < PXT; ++i) {
                            m[i] += k * r[i + 2 * HH - uu];
                            v[i] += k2 * q[i + 2 * HH - uu];
                        }
                    }
                }
                uint8_t foot[PXT];
#pragma unroll
                for (int i = 0; i < PXT; ++i) foot[i] = 0;
                for (int vv = 0; vv < K; ++vv)
#pragma unroll
                    for (int i = 0; i < PXT; ++i) foot[i] |= Mr[(ly + vv) * BW + lx0 + i];
#pragma unroll
                for (int i = 0; i < PXT; ++i) {
                    const int X = tx0 + lx0 + i;
                    if (X >= L) continue;
                    const int64_t o = org + (int64_t)Y * P + X;
                    const bool edge = X < HH || X > L - 1 - HH || Y < HH || Y > L - 1 - HH;
                    const uint8_t dm = gld(fr.sci_mask + o) | (edge ? ARGUS_EDGE : 0u) |
                                       ((!edge && foot[i]) ? ARGUS_FOOT : 0u);
                    float dval = 0.f, vval = 0.f;
                    if (dm == 0) {
                        const float sv = gld(fr.sci_var + o);
                        dval = gld(fr.sci + o) - (float)((double)m[i] + (double)bg);
                        vval = sv + v[i];
                        const float tot = sv + gld(fr.ref_var + o);
                        if (tot > 0.f) {
                            c2 += (double)dval * (double)dval / (double)tot;
                            cnt += 1.0;
                        }
                    }
                    const int64_t oo = (int64_t)Y * L + X;
                    dout[oo] = dval;
                    vout[oo] = vval;
                    mout[oo] = dm;
                }
            }
            __syncthreads();
        }
    }
    // ---- detection map of the cutout (off-cutout neighbours are -inf) ----
    __threadfence_block();
    __syncthreads();
    float (*s)[512 + 4] = (float (*)[512 + 4])lds;
    int ncand = 0;
    for (int y0 = 0; y0 < L; y0 += DROWS) {
        for (int i = tid; i < (DROWS + 2) * (L + 2); i += NTHR) {
            int row = i / (L + 2), cc = i % (L + 2);
            int X = cc - 1, Y = y0 - 1 + row;
            float sn = -__builtin_inff();
            if (X >= 0 && X < L && Y >= 0 && Y < L) {
                int64_t oo = (int64_t)Y * L + X;
                float V = vout[oo];
                sn = (mout[oo] != 0 || !(V > 0.f)) ? 0.f : dout[oo] * __builtin_amdgcn_rsqf(V);
            }
            s[row][cc] = sn;
        }
        __syncthreads();
        for (int i = tid; i < DROWS * L; i += NTHR) {
            const int rr = i / L, X = i % L, Y = y0 + rr;
            if (Y >= L) continue;
            const float cval = s[rr + 1][X + 1];
            const bool det = cval >= a.thr;
            bool cand = det && cval > s[rr][X] && cval > s[rr][X + 1] && cval > s[rr][X + 2] &&
                        cval > s[rr + 1][X];
            cand = cand && cval >= s[rr + 1][X + 2] && cval >= s[rr + 2][X] &&
                   cval >= s[rr + 2][X + 1] && cval >= s[rr + 2][X + 2];
            a.det[cu.out_offset + (int64_t)Y * L + X] = (det ? ARGUS_DET : 0u) | (cand ? ARGUS_CAND : 0u);
            ncand += cand;
        }
        __syncthreads();
    }
    // ---- per-cutout sums, fixed order ----
    __shared__ double red[3][4];
    for (int off = 32; off > 0; off >>= 1) {
        c2 += __shfl_xor(c2, off);
        cnt += __shfl_xor(cnt, off);
        ncand += __shfl_xor(ncand, off);
    }
    if (lane == 0) { red[0][wave] = c2; red[1][wave] = cnt; red[2][wave] = (double)ncand; }
    __syncthreads();
    if (tid == 0) {
        a.chi2[c] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        a.n_cands[c] = (int32_t)(red[2][0] + red[2][1] + red[2][2] + red[2][3]);
    }
    __syncthreads();
}

template <int HH, int TILE, int PREC>
__global__ __launch_bounds__(NTHR, 2) void batch_kernel(BatchArgs a) {
    extern __shared__ float lds[];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1);
        __syncthreads();
        const int it = s_item;
        __syncthreads();
        if (it >= a.n) break;                       // every wave reaches this exit
        process_cutout<HH, TILE, PREC>(a, a.order[it], lds);
    }
}

__global__ void queue_reset_kernel(int32_t *q) { *q = 0; }

inline int ilog2(int64_t v) {
    int r = 0;
    while (v > 1) { v >>= 1; ++r; }
    return r;
}

// candidates: subtraction tile height x workgroups per CU
constexpr int N_CAND = 6;
constexpr int CAND_TILE[N_CAND] = {16, 16, 16, 32, 32, 32};
constexpr int CAND_WPC[N_CAND] = {1, 2, 3, 1, 2, 3};

template <int HH, int TILE, int PREC>
int batch_launch_t(argus_ctx *ctx, const BatchArgs &ba, int wg_per_cu, hipStream_t st) {
    size_t lds = BatchLds<HH, TILE>::bytes(ba.nplanes);
    ARGUS_HIP_CHECK(ctx, hipFuncSetAttribute((const void *)batch_kernel<HH, TILE, PREC>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int cus = 0;
    ARGUS_HIP_CHECK(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    int grid = std::max(1, std::min(cus * wg_per_cu, ba.n));
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(1), 0, st, ba.queue);
    hipLaunchKernelGGL((batch_kernel<HH, TILE, PREC>), dim3(grid), dim3(NTHR), lds, st, ba);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

int batch_launch(argus_ctx *ctx, const BatchArgs &ba, int h, int prec, int cand, hipStream_t st) {
    const int tile = CAND_TILE[cand], wpc = CAND_WPC[cand];
#define ARGUS_BH(HH)                                                                          \
    case HH:                                                                                  \
        if (prec == ARGUS_FP64)                                                               \
            return tile == 16 ? batch_launch_t<HH, 16, ARGUS_FP64>(ctx, ba, wpc, st)          \
                              : batch_launch_t<HH, 32, ARGUS_FP64>(ctx, ba, wpc, st);         \
        return tile == 16 ? batch_launch_t<HH, 16, ARGUS_FP32>(ctx, ba, wpc, st)              \
                          : batch_launch_t<HH, 32, ARGUS_FP32>(ctx, ba, wpc, st);
    switch (h) {
        ARGUS_BH(4) ARGUS_BH(5) ARGUS_BH(6) ARGUS_BH(7) ARGUS_BH(8) ARGUS_BH(9) ARGUS_BH(10)
        default: return argus_fail(ctx, ARGUS_ESHAPE, "batch half width %d not in 4..10", h);
    }
#undef ARGUS_BH
}

}  // namespace

extern "C" {

int argus_batch_plan(argus_ctx *ctx, const argus_kernel_spec *spec, const argus_cutout *cutouts,
                     int n_cutouts, const int32_t *frame_widths, const int32_t *frame_heights,
                     int n_frames, argus_batch **out) {
    if (!ctx || !out) return ARGUS_EINVAL;
    ctx->err.clear();
    *out = nullptr;
    int nu, ns;
    int rc = argus_kernel_dims(spec, &nu, &ns);
    if (rc) return argus_fail(ctx, rc, "argus_batch_plan: bad kernel spec");
    if (spec->spatial_degree != 0 || spec->mode != ARGUS_FIT_GLOBAL ||
        (spec->precision != ARGUS_FP32 && spec->precision != ARGUS_FP64))
        return argus_fail(ctx, ARGUS_ESHAPE, "batch fits use degree 0, GLOBAL, FP32 or FP64");
    if (spec->half_width < 4 || spec->half_width > 10)
        return argus_fail(ctx, ARGUS_ESHAPE, "batch half width %d not in 4..10", spec->half_width);
    if (n_cutouts < 1 || !cutouts || n_frames < 1 || !frame_widths || !frame_heights)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_batch_plan: empty or null tables");
    const int h = spec->half_width;
    for (int i = 0; i < n_cutouts; ++i) {
        const argus_cutout &c = cutouts[i];
        if (c.frame < 0 || c.frame >= n_frames)
            return argus_fail(ctx, ARGUS_EINVAL, "cutout %d: frame %d out of range", i, c.frame);
        if (c.side < 2 * h + 2 || c.side > 512)
            return argus_fail(ctx, ARGUS_ESHAPE, "cutout %d: side %d not in %d..512", i, c.side, 2 * h + 2);
        if (c.x0 < 0 || c.y0 < 0 || c.x0 + c.side > frame_widths[c.frame] ||
            c.y0 + c.side > frame_heights[c.frame])
            return argus_fail(ctx, ARGUS_ESHAPE, "cutout %d leaves its frame", i);
        if (c.out_offset < 0) return argus_fail(ctx, ARGUS_EINVAL, "cutout %d: negative offset", i);
    }
    argus_batch *b = new argus_batch();
    for (int i = 0; i < n_cutouts; ++i) b->area += (int64_t)cutouts[i].side * cutouts[i].side;
    b->n = n_cutouts;
    b->n_frames = n_frames;
    b->n_unk = nu;
    b->h = h;
    b->spec = *spec;
    b->nb = argus_nbasis(spec);
    b->nplanes = argus_nplanes(spec);
    b->widths.assign(frame_widths, frame_widths + n_frames);
    b->heights.assign(frame_heights, frame_heights + n_frames);
    // planes to waves (same balancing as the frame fit)
    {
        int cost[ARGUS_MAX_PLANES], load[4] = {0, 0, 0, 0}, nin[4] = {0, 0, 0, 0};
        int p = 0;
        for (int g = 0; g < spec->n_gauss; ++g)
            for (int i = 0; i <= spec->degree[g]; ++i, ++p) cost[p] = 2 + spec->degree[g] - i;
        for (int w = 0; w < 4; ++w)
            for (int j = 0; j < 4; ++j) b->plist[w][j] = -1;
        bool used[ARGUS_MAX_PLANES] = {};
        for (int k = 0; k < b->nplanes; ++k) {
            int best = -1;
            for (int q = 0; q < b->nplanes; ++q)
                if (!used[q] && (best < 0 || cost[q] > cost[best])) best = q;
            int w = -1;
            for (int c = 0; c < 4; ++c)
                if (nin[c] < 4 && (w < 0 || load[c] < load[w])) w = c;
            used[best] = true;
            b->plist[w][nin[w]++] = (int8_t)best;
            load[w] += cost[best];
        }
    }
    // largest cutouts first; ties by index (deterministic)
    std::vector<int32_t> order(n_cutouts);
    for (int i = 0; i < n_cutouts; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return cutouts[a].side > cutouts[c].side; });
    size_t bc = (size_t)n_cutouts * sizeof(argus_cutout), bo = (size_t)n_cutouts * 4,
           bf = (size_t)n_frames * sizeof(argus_frame);
    size_t off_o = (bc + 255) & ~(size_t)255, off_f = (off_o + bo + 255) & ~(size_t)255,
           off_q = (off_f + bf + 255) & ~(size_t)255, off_t = off_q + 256;
    if (hipMalloc(&b->dev, off_t + sizeof(BasisTables)) != hipSuccess) {
        delete b;
        return argus_fail(ctx, ARGUS_ENOMEM, "batch tables");
    }
    b->d_cuts = (argus_cutout *)b->dev;
    b->d_order = (int32_t *)((char *)b->dev + off_o);
    b->d_frames = (argus_frame *)((char *)b->dev + off_f);
    b->d_queue = (int32_t *)((char *)b->dev + off_q);
    b->d_tables = (BasisTables *)((char *)b->dev + off_t);
    if (hipMemcpy(b->d_cuts, cutouts, bc, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_order, order.data(), bo, hipMemcpyHostToDevice) != hipSuccess ||
        hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess) {
        argus_batch_destroy(b);
        return argus_fail(ctx, ARGUS_EHIP, "batch setup failed");
    }
    if ((rc = launch_basis_tables_to(ctx, spec, b->d_tables))) {
        argus_batch_destroy(b);
        return rc;
    }
    // the basis tables must be complete before the private stream reads them
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
        argus_batch_destroy(b);
        return argus_fail(ctx, ARGUS_EHIP, "batch setup sync failed");
    }
    *out = b;
    return ARGUS_OK;
}

int argus_batch_run(argus_ctx *ctx, argus_batch *b, const argus_frame *frames, float threshold,
                    float *diff, float *diff_var, uint8_t *diff_mask, uint8_t *det_mask,
                    double *coeffs, double *chi2, int64_t *n_fit, int32_t *status,
                    int32_t *n_cands) {
    if (!ctx || !b || !frames) return ARGUS_EINVAL;
    ctx->err.clear();
    if (!diff || !diff_var || !diff_mask || !det_mask || !coeffs || !chi2 || !n_fit || !status ||
        !n_cands)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_batch_run: null output");
    for (int f = 0; f < b->n_frames; ++f) {
        const argus_frame &fr = frames[f];
        if (!fr.ref || !fr.ref_var || !fr.ref_mask || !fr.sci || !fr.sci_var || !fr.sci_mask)
            return argus_fail(ctx, ARGUS_EINVAL, "frame %d: null plane", f);
        if (fr.width != b->widths[f] || fr.height != b->heights[f] || fr.pitch < fr.width)
            return argus_fail(ctx, ARGUS_ESHAPE, "frame %d does not match the plan", f);
    }
    const void *outs[9] = {diff, diff_var, diff_mask, det_mask, coeffs, chi2, n_fit, status, n_cands};
    bool same = b->exec && b->thr == threshold && (int)b->frames.size() == b->n_frames;
    for (int i = 0; same && i < 9; ++i) same = b->outs[i] == outs[i];
    for (int f = 0; same && f < b->n_frames; ++f)
        same = memcmp(&b->frames[f], &frames[f], sizeof(argus_frame)) == 0;
    // order the private stream after the caller's stream
    ARGUS_HIP_CHECK(ctx, hipEventRecord(b->ev_in, ctx->stream));
    ARGUS_HIP_CHECK(ctx, hipStreamWaitEvent(b->stream, b->ev_in, 0));
    if (!same) {
        ARGUS_HIP_CHECK(ctx, hipMemcpyAsync(b->d_frames, frames, (size_t)b->n_frames * sizeof(argus_frame),
                                            hipMemcpyHostToDevice, b->stream));
        ARGUS_HIP_CHECK(ctx, hipStreamSynchronize(b->stream));
        BatchArgs ba;
        ba.frames = b->d_frames; ba.cuts = b->d_cuts; ba.order = b->d_order; ba.queue = b->d_queue;
        ba.tab = b->d_tables; ba.n = b->n; ba.nb = b->nb; ba.nplanes = b->nplanes; ba.n_unk = b->n_unk;
        memcpy(ba.plist, b->plist, sizeof ba.plist);
        ba.thr = threshold;
        ba.diff = diff; ba.dvar = diff_var; ba.dmask = diff_mask; ba.det = det_mask;
        ba.coeffs = coeffs; ba.chi2 = chi2; ba.n_fit = n_fit; ba.status = status; ba.n_cands = n_cands;
        if (b->choice < 0) {
            // autotune: the context's cache (device, HIP runtime, kernel, half
            // width, precision, size bucket), else time each candidate once on
            // these inputs and store the outcome
            char kb[160];
            snprintf(kb, sizeof kb, ";kernel=batch;h=%d;prec=%d;log2n=%d;log2area=%d", b->h,
                     b->spec.precision, ilog2(b->n), ilog2(b->area));
            const std::string key = argus_tune_device_key(ctx) + kb;
            const argus_ctx::Tuned *t = argus_tune_lookup(ctx, key);
            if (t && (int)t->ms.size() == N_CAND) {
                b->choice = t->choice;
                b->cand_ms = t->ms;
                b->from_cache = 1;
            } else {
                hipEvent_t e0, e1;
                ARGUS_HIP_CHECK(ctx, hipEventCreate(&e0));
                ARGUS_HIP_CHECK(ctx, hipEventCreate(&e1));
                float best = 1e30f;
                b->cand_ms.assign(N_CAND, 0.f);
                for (int cand = 0; cand < N_CAND; ++cand) {
                    ARGUS_HIP_CHECK(ctx, hipEventRecord(e0, b->stream));
                    int rc = batch_launch(ctx, ba, b->h, b->spec.precision, cand, b->stream);
                    if (rc) return rc;
                    ARGUS_HIP_CHECK(ctx, hipEventRecord(e1, b->stream));
                    ARGUS_HIP_CHECK(ctx, hipEventSynchronize(e1));
                    float ms = 0.f;
                    ARGUS_HIP_CHECK(ctx, hipEventElapsedTime(&ms, e0, e1));
                    b->cand_ms[cand] = ms;
                    if (ms < best) { best = ms; b->choice = cand; }
                }
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                argus_tune_store(ctx, key, b->choice, b->cand_ms);
                b->from_cache = 0;
            }
            b->tuned_ms = b->cand_ms[b->choice];
            b->n_cand = N_CAND;
        }
        if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
        if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
        ARGUS_HIP_CHECK(ctx, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        int rc = batch_launch(ctx, ba, b->h, b->spec.precision, b->choice, b->stream);
        hipGraph_t g = nullptr;
        hipError_t ec = hipStreamEndCapture(b->stream, &g);
        if (rc) return rc;
        if (ec != hipSuccess) return argus_fail(ctx, ARGUS_EHIP, "graph capture failed");
        b->graph = g;
        ARGUS_HIP_CHECK(ctx, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->frames.assign(frames, frames + b->n_frames);
        memcpy(b->outs, outs, sizeof outs);
        b->thr = threshold;
    }
    argus_time_begin(ctx);
    ARGUS_HIP_CHECK(ctx, hipGraphLaunch(b->exec, b->stream));
    ARGUS_HIP_CHECK(ctx, hipEventRecord(b->ev_out, b->stream));
    ARGUS_HIP_CHECK(ctx, hipStreamWaitEvent(ctx->stream, b->ev_out, 0));
    argus_time_end(ctx, "batch");
    return ARGUS_OK;
}

int argus_batch_tuning(const argus_batch *b, float *cand_ms, int capacity, int *n_candidates,
                       int *from_cache) {
    if (!b || capacity < 0 || (capacity > 0 && !cand_ms)) return ARGUS_EINVAL;
    const int n = (int)b->cand_ms.size();
    for (int i = 0; i < n && i < capacity; ++i) cand_ms[i] = b->cand_ms[i];
    if (n_candidates) *n_candidates = n;
    if (from_cache) *from_cache = b->from_cache;
    return ARGUS_OK;
}

int argus_batch_candidate(int index, int *tile_rows, int *wg_per_cu) {
    if (index < 0 || index >= N_CAND) return ARGUS_EINVAL;
    if (tile_rows) *tile_rows = CAND_TILE[index];
    if (wg_per_cu) *wg_per_cu = CAND_WPC[index];
    return ARGUS_OK;
}

int argus_batch_info(const argus_batch *b, int *choice, float *ms, int *n_candidates) {
    if (!b) return ARGUS_EINVAL;
    if (choice) *choice = b->choice;
    if (ms) *ms = b->tuned_ms;
    if (n_candidates) *n_candidates = b->n_cand;
    return ARGUS_OK;
}

void argus_batch_destroy(argus_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    if (b->dev) (void)hipFree(b->dev);
    delete b;
}

}  // extern "C"
