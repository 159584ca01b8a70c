// Wave-specialised form of the fused basis convolution + moment accumulation
// for whole frames: NWC convolution waves (row filters, column filters,
// fit-set weights) and NWM MFMA waves per workgroup.  The convolution of output row y and the moments of row y-1 run at
// the same time on double-buffered operand tables, so every SIMD holds one
// wave of each kind and its VALU and matrix pipes overlap; there is one
// barrier per input row.
//
// The operand tables are k-major (c[k][p]) so that a lane's operands of
// four consecutive MFMA steps are one 16-byte LDS read; the per-row sums
// take the pixels in a different order than fit_wave, otherwise the
// arithmetic (filters, products, FP64 flushes) is the same.
#pragma once
#include "fit_accum.h"

namespace argus_fit {


template <int D, int HH>
struct FitLds8 {
    static constexpr int K = 2 * HH + 1;
    static constexpr int IN = SW + 2 * HH;               // input row length
    static constexpr int INP = (IN + 3) & ~3;
    float *rowbuf, *inrow, *cvec0, *wx0, *wsx0;
    double *wxd0, *wsxd0;
    uint8_t *minrow;
    static constexpr int CKM = SW + 4;                   // k-major row stride of c
    // buffer b (0/1) of each double-buffered table (no pointer arrays: a
    // runtime index into one would place it in scratch)
    __device__ float *cvec(int b) const { return cvec0 + b * (32 * CKM); }
    __device__ float *wx(int b) const { return wx0 + b * (FitShape<D>::NA * SW); }
    __device__ float *wsx(int b) const { return wsx0 + b * (FitShape<D>::NRA * SW); }
    __device__ double *wxd(int b) const { return wxd0 + b * (FitShape<D>::NA * SW); }
    __device__ double *wsxd(int b) const { return wsxd0 + b * (FitShape<D>::NRA * SW); }
    __host__ __device__ static size_t bytes(int nplanes) {
        using S = FitShape<D>;
        size_t w = (size_t)nplanes * K * SW + 2 * INP + 2 * 32 * CKM + 2 * (S::NA + S::NRA) * SW;
        size_t b = w * 4 + 16 + (size_t)2 * (S::NA + S::NRA) * SW * 8 + 2 * INP + 16;
        size_t rhs = (size_t)16 * S::NR * 32 * 8 + 256;   // end-of-kernel reuse of rowbuf
        return (b > rhs ? b : rhs) + 64;
    }
    __device__ FitLds8(float *lds, int nplanes) {
        using S = FitShape<D>;
        rowbuf = lds;                                   // [NPL][K][SW]: thread-private columns
        inrow = rowbuf + (size_t)nplanes * K * SW;      // [2][INP] double-buffered input row
        cvec0 = inrow + 2 * INP;                        // [2][32][CKM] k-major
        wx0 = cvec0 + 2 * 32 * CKM;                     // [2][NA][SW]
        wsx0 = wx0 + 2 * S::NA * SW;                    // [2][NRA][SW]
        // every region above is a multiple of 16 bytes long (INP, SW, CKM are
        // multiples of 4): no integer round trip, which would turn the LDS
        // pointers into generic ones
        wxd0 = (double *)(wsx0 + 2 * S::NRA * SW);
        wsxd0 = wxd0 + 2 * S::NA * SW;
        minrow = (uint8_t *)(wsxd0 + 2 * S::NRA * SW);  // [2][INP] ref mask != 0
    }
};

// Wave W of the workgroup: W < NWC convolves (its planes from plist, or
// plist8 with 8 convolution waves; wave 0 also stages the fit-set weights),
// W >= NWC accumulates the tasks W - NWC, W - NWC + NWM, ... on MFMA.  Both
// roles walk the same rows and meet at the same barriers.
template <int D, int HH, int W, int PREC, int NWC, int NWM>
__device__ void fit_wave8(const FitArgs &a, float *lds, int sx_begin, int sx_end, int ry0,
                          int ry1, bool active, double *part) {
    using S = FitShape<D>;
    using L = FitLds8<D, HH>;
    constexpr int K = L::K;
    constexpr bool CONV = W < NWC;
    constexpr int MW = CONV ? 0 : W - NWC;
    constexpr int NPW = NWC == 4 ? 4 : 2;                // plane slots per convolution wave
    constexpr int NTH = 64 * (NWC + NWM);
    constexpr int PXW = SW / NWM, PXH = PXW / 2;         // rhs pixels per wave and half-wave
    auto plane = [&](int j) -> int {
        if constexpr (NWC == 4) return a.plist[W < 4 ? W : 0][j];
        else return a.plist8[W < 8 ? W : 0][j];
    };
    const int tid = threadIdx.x, lane = tid & 63;
    const int NPL = a.nplanes;
    L l(lds, NPL);
    double *rhsbuf = (double *)lds;

    WaveGram<D, MW, PREC, NWM> gram;
    double RF[S::NR];
    if constexpr (!CONV) {
        gram.zero();
#pragma unroll
        for (int i = 0; i < S::NR; ++i) RF[i] = 0.0;
    }
    int count = 0;

    // convolution waves: this wave's planes (wave-uniform)
    int k0[NPW], nk[NPW];
#pragma unroll
    for (int j = 0; j < NPW; ++j) {
        k0[j] = 0;
        nk[j] = 0;
        if constexpr (CONV) {
            const int p = plane(j);
            if (p >= 0) {
                for (int k = 0; k < a.nb; ++k)
                    if (a.tab->kpl[k] == p) {
                        if (nk[j] == 0) k0[j] = k;
                        ++nk[j];
                    }
            }
            k0[j] = __builtin_amdgcn_readfirstlane(k0[j]);
            nk[j] = __builtin_amdgcn_readfirstlane(nk[j]);
        }
    }
    const float g0 = (lane & 15) < a.nb ? a.tab->gam[lane & 15] : 0.f;
    const float g1 = 16 + (lane & 15) < a.nb ? a.tab->gam[16 + (lane & 15)] : 0.f;
    const float gk = (lane & 31) < a.nb ? a.tab->gam[lane & 31] : 0.f;  // rhs fix-up
    const int nstrips = active ? (sx_end - sx_begin + SW - 1) / SW : 1;
    for (int strip = 0; strip < nstrips; ++strip) {
        const int sx0 = sx_begin + strip * SW, sx1 = min(sx0 + SW, sx_end);
        const double xtd = (double)(sx0 + lane) * a.sx - (a.sx != 0.0 ? 1.0 : 0.0);
        const float xt = (float)xtd;
        const int64_t P = a.pitch;
        // Input rows are staged two ahead: row yy+1 goes to LDS during row yy.
        // The prefetches only load (from clamped addresses); the in-frame
        // selects happen where the values are used, a row later, so the loads
        // stay in flight for a whole row instead of being waited for at once.
        float pr = 0.f;
        uint8_t pm = 0;
        bool pin = false;
        float p_s = 0.f, p_sv = 0.f, p_rv = 0.f;
        uint8_t p_sm = 1;
        bool pok = false;
        const int Xin = sx0 - HH + tid;
        const bool in_x = tid < L::IN && Xin >= 0 && Xin < a.W;
        const int Xc = in_x ? Xin : (Xin < 0 ? 0 : a.W - 1);
        auto fetch_in = [&](int yy) {
            if (tid < L::IN) {
                pr = a.ref[(int64_t)yy * P + Xc];
                pm = a.rmask[(int64_t)yy * P + Xc];
                pin = in_x;
            }
        };
        const bool lane_ok = sx0 + lane < sx1;
        const int64_t xw = lane_ok ? sx0 + lane : sx0;
        auto fetch_w = [&](int y) {
            if (W == 0) {
                pok = lane_ok && y >= ry0 && y < ry1;
                const int yc = y < ry1 ? y : ry1 - 1;
                const int64_t o = (int64_t)yc * P + xw;
                p_s = a.sci[o];
                p_sv = a.svar[o];
                p_rv = a.rvar[o];
                p_sm = a.smask[o];
            }
        };
        auto stage = [&](int b) {
            if (tid < L::IN) {
                l.inrow[b * L::INP + tid] = pin ? pr : 0.f;
                l.minrow[b * L::INP + tid] = (pin && pm != 0) ? 1 : 0;
            }
        };
        uint32_t hist = 0;                 // bit j: input row yy-j has a flagged pixel in reach
        const int ystart = ry0 - HH;
        const int yend = active ? ry1 + HH : ystart;
        if constexpr (CONV) {
            if (active) {
                fetch_in(ystart);
                stage(ystart & 1);
                if (ystart + 1 < yend) fetch_in(ystart + 1);
                fetch_w(ry0);
            }
        }
        __syncthreads();
        // one extra step drains the last output row into the moments
        for (int yy = ystart; yy <= yend; ++yy) {
            const int buf = yy & 1;
            if constexpr (CONV) {
                if (yy < yend) {
                    // stage input row yy+1, prefetch row yy+2
                    if (yy + 1 < yend) stage(buf ^ 1);
                    if (yy + 2 < yend) fetch_in(yy + 2);
                    const float w_s = p_s, w_sv = p_sv, w_rv = p_rv;
                    const uint8_t w_sm = pok ? p_sm : 1;
                    const bool outrow = yy >= ry0 + HH;
                    if (outrow) fetch_w(yy + 1 - HH);
                    const int slot = yy % K;
                    {
                        float win[K];
                        const float *ir = l.inrow + buf * L::INP + lane;
#pragma unroll
                        for (int uu = 0; uu < K; ++uu) win[uu] = ir[2 * HH - uu];
#pragma unroll
                        for (int j = 0; j < NPW; ++j) {
                            const int p = plane(j);
                            if (p >= 0) {
                                const float *f = &a.tab->rowf[p][0];
                                float acc = 0.f;
#pragma unroll
                                for (int uu = 0; uu < K; ++uu) acc += uload(f + uu) * win[uu];
                                l.rowbuf[((size_t)p * K + slot) * SW + lane] = acc;
                            }
                        }
                        if (W == 0) {
                            const uint8_t *mr = l.minrow + buf * L::INP + lane;
                            uint8_t m = 0;
#pragma unroll
                            for (int uu = 0; uu < K; ++uu) m |= mr[uu];
                            hist = (hist << 1) | (m ? 1u : 0u);
                        }
                    }
                    if (outrow) {
                        // column filters: rows y-h..y+h sit in slots (yy+1 .. yy+K) mod K
                        const int s0 = (yy + 1) % K;
                        float *cv = l.cvec(buf);
#pragma unroll
                        for (int j = 0; j < NPW; ++j) {
                            const int p = plane(j);
                            if (p >= 0) {
                                float t[K];
#pragma unroll
                                for (int jj = 0; jj < K; ++jj) {
                                    int sl = s0 + jj;
                                    sl -= sl >= K ? K : 0;
                                    t[jj] = l.rowbuf[((size_t)p * K + sl) * SW + lane];
                                }
#pragma unroll
                                for (int q = 0; q < 5; ++q) {
                                    if (q < nk[j]) {
                                        const float *f = &a.tab->colf[k0[j] + q][0];
                                        float acc = 0.f;
#pragma unroll
                                        for (int jj = 0; jj < K; ++jj)
                                            acc += uload(f + 2 * HH - jj) * t[jj];
                                        cv[(k0[j] + q) * L::CKM + lane] = acc;
                                    }
                                }
                            }
                        }
                        if (W == 0) {
                            const bool foot = (hist & ((1u << K) - 1u)) != 0;
                            const float tot = w_sv + w_rv;
                            float w = 0.f;
                            if (w_sm == 0 && !foot && tot > 0.f) {
                                w = 1.0f / tot;
                                ++count;
                            }
                            float xp = 1.f;
                            double xpd = 1.0;
#pragma unroll
                            for (int e = 0; e < S::NA; ++e) {
                                l.wx(buf)[e * SW + lane] = w * xp;
                                if (PREC == ARGUS_FP64) l.wxd(buf)[e * SW + lane] = (double)w * xpd;
                                if (e < S::NRA) l.wsx(buf)[e * SW + lane] = w * w_s * xp;
                                if (PREC == ARGUS_FP64 && e < S::NRA)
                                    l.wsxd(buf)[e * SW + lane] = (double)w * (double)w_s * xpd;
                                xp *= xt;
                                xpd *= xtd;
                            }
                        }
                    }
                }
            } else {
                // moments of output row y = yy - 1 - h, written during the previous step
                const int y = yy - 1 - HH;
                if (yy - 1 >= ry0 + HH && yy - 1 < yend) {
                    const int pb = buf ^ 1;
                    double ypw[2 * D + 1];
                    {
                        const double yt = (double)y * a.sy - (a.sy != 0.0 ? 1.0 : 0.0);
                        double yp = 1.0;
#pragma unroll
                        for (int b = 0; b <= 2 * D; ++b) { ypw[b] = yp; yp *= yt; }
                    }
                    gram.row_km(l.cvec(pb), l.wx(pb), l.wxd(pb), ypw, lane, g0, g1);
                    const float *cv = l.cvec(pb);
                    const int k = lane & 31, half = lane >> 5;
                    if constexpr (PREC == ARGUS_FP64) {
                        double ra[S::NRA];
#pragma unroll
                        for (int e = 0; e < S::NRA; ++e) ra[e] = 0.0;
#pragma unroll
                        for (int i = 0; i < PXH; ++i) {
                            const int px = MW * PXW + half * PXH + i;
                            const double c = (double)cv[k * L::CKM + px] + (double)gk * (double)cv[px];
#pragma unroll
                            for (int e = 0; e < S::NRA; ++e) ra[e] += l.wsxd(pb)[e * SW + px] * c;
                        }
#pragma unroll
                        for (int e = 0; e < S::NRA; ++e)
#pragma unroll
                            for (int b = 0; b <= D; ++b)
                                if (e + b <= D) RF[qidx(e, b, D)] += ypw[b] * ra[e];
                    } else {
                        float ra[S::NRA];
#pragma unroll
                        for (int e = 0; e < S::NRA; ++e) ra[e] = 0.f;
#pragma unroll
                        for (int i = 0; i < PXH; ++i) {
                            const int px = MW * PXW + half * PXH + i;
                            const float c = cv[k * L::CKM + px] + gk * cv[px];
#pragma unroll
                            for (int e = 0; e < S::NRA; ++e) ra[e] += l.wsx(pb)[e * SW + px] * c;
                        }
#pragma unroll
                        for (int e = 0; e < S::NRA; ++e)
#pragma unroll
                            for (int b = 0; b <= D; ++b)
                                if (e + b <= D) RF[qidx(e, b, D)] += ypw[b] * (double)ra[e];
                    }
                }
            }
            __syncthreads();
        }
    }
    // partials: moments (MFMA waves), rhs pieces through LDS, fit-set count
    if constexpr (!CONV) {
        gram.store(part, lane);
        const int k = lane & 31, half = lane >> 5;
#pragma unroll
        for (int i = 0; i < S::NR; ++i) rhsbuf[((MW * 2 + half) * S::NR + i) * 32 + k] = RF[i];
    }
    if constexpr (W == 0) {
        double c = (double)count;
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
        if (lane == 0) part[(size_t)S::NQ * 768 + S::NR * 32] = c;
    }
    __syncthreads();
    for (int it = tid; it < S::NR * 32; it += NTH) {
        double s = 0.0;
        for (int q = 0; q < 2 * NWM; ++q) s += rhsbuf[q * S::NR * 32 + it];
        part[(size_t)S::NQ * 768 + it] = s;
    }
}

template <int D, int HH, int PREC, int NWC, int NWM, int W>
__device__ __forceinline__ void fit_dispatch8(int w, const FitArgs &a, float *lds, int sx0, int sx1,
                                              int ry0, int ry1, bool active, double *part) {
    if constexpr (W < NWC + NWM) {
        if (w == W)
            fit_wave8<D, HH, W, PREC, NWC, NWM>(a, lds, sx0, sx1, ry0, ry1, active, part);
        else
            fit_dispatch8<D, HH, PREC, NWC, NWM, W + 1>(w, a, lds, sx0, sx1, ry0, ry1, active, part);
    }
}

template <int D, int HH, int PREC, int NWC, int NWM>
__global__ __launch_bounds__(64 * (NWC + NWM)) void fit_accum8_kernel(FitArgs a) {
    extern __shared__ __align__(16) float lds[];
    constexpr int NTH = 64 * (NWC + NWM);
    const int tid = threadIdx.x;
    // workgroup -> region, strip, row chunk
    const int s = blockIdx.x % a.spt, rx = blockIdx.x / a.spt;
    const int rc = blockIdx.y % a.rchunks, ry = blockIdx.y / a.rchunks;
    const int rx0 = (int)((int64_t)rx * a.W / a.RX), rx1 = (int)((int64_t)(rx + 1) * a.W / a.RX);
    const int ry0g = (int)((int64_t)ry * a.H / a.RY), ry1g = (int)((int64_t)(ry + 1) * a.H / a.RY);
    const int ix0 = max(rx0, HH), ix1 = min(rx1, a.W - HH);
    const int iy0 = max(ry0g, HH), iy1 = min(ry1g, a.H - HH);
    const int sx0 = ix0 + s * SW, sx1 = min(sx0 + SW, ix1);
    const int rows = max(iy1 - iy0, 0);
    const int rh = (rows + a.rchunks - 1) / a.rchunks;
    const int ry0 = iy0 + rc * rh, ry1 = min(ry0 + rh, iy1);
    const bool active = sx0 < sx1 && ry0 < ry1;    // otherwise the partial is all zeros
    const int pid = ((ry * a.RX + rx) * a.rchunks + rc) * a.spt + s;
    double *part = a.partials + (size_t)pid * a.stride;
    // constant tail of c: 1 at index nb (background), zeros after, both buffers
    FitLds8<D, HH> L(lds, a.nplanes);
    for (int i = tid; i < 2 * 32 * FitLds8<D, HH>::CKM; i += NTH) {
        const int k = (i / FitLds8<D, HH>::CKM) % 32;
        if (k >= a.nb) L.cvec0[i] = (k == a.nb) ? 1.f : 0.f;
    }
    fit_dispatch8<D, HH, PREC, NWC, NWM, 0>(tid >> 6, a, lds, sx0, sx1, ry0, ry1, active, part);
}

// Launch fit_accum8_kernel<D, h, PREC, ...> with its dynamic LDS size: FP32
// runs 8 convolution + 8 MFMA waves (two tasks each, so every wave fits in
// 128 registers and each SIMD holds four waves); the FP64 and BF16x3 forms,
// whose MFMA waves need more registers, run 4 + 4.
template <int PREC>
int fit_accum8_launch(argus_ctx *ctx, const FitArgs &fa, int D, dim3 grid) {
    constexpr int NW = PREC == ARGUS_FP32 ? 8 : 4;
    hipError_t err = hipSuccess;
    bool ok = false;
#define ARGUS_FH(DD, HH)                                                                   \
    if (D == DD && fa.h == HH) {                                                           \
        size_t lds = FitLds8<DD, HH>::bytes(fa.nplanes);                                   \
        err = hipFuncSetAttribute((const void *)fit_accum8_kernel<DD, HH, PREC, NW, NW>,   \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        if (err == hipSuccess)                                                             \
            hipLaunchKernelGGL((fit_accum8_kernel<DD, HH, PREC, NW, NW>), grid,            \
                               dim3(64 * 2 * NW), lds, ctx->stream, fa);                   \
        ok = true;                                                                         \
    }
#define ARGUS_FD(DD)                                                                       \
    ARGUS_FH(DD, 1) ARGUS_FH(DD, 2) ARGUS_FH(DD, 3) ARGUS_FH(DD, 4) ARGUS_FH(DD, 5)         \
    ARGUS_FH(DD, 6) ARGUS_FH(DD, 7) ARGUS_FH(DD, 8) ARGUS_FH(DD, 9) ARGUS_FH(DD, 10)        \
    ARGUS_FH(DD, 11) ARGUS_FH(DD, 12) ARGUS_FH(DD, 13) ARGUS_FH(DD, 14) ARGUS_FH(DD, 15)
    ARGUS_FD(0)
    ARGUS_FD(1)
    ARGUS_FD(2)
#undef ARGUS_FD
#undef ARGUS_FH
    if (!ok) return argus_fail(ctx, ARGUS_ESHAPE, "unsupported degree %d / half width %d", D, fa.h);
    ARGUS_HIP_CHECK(ctx, err);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

}  // namespace argus_fit
