// Wave-specialised form of the fused basis convolution + moment accumulation
// for whole frames: 8 convolution waves (row filters, column filters,
// fit-set weights) and NWM MFMA waves per workgroup.  The convolution of
// output row y and the moments of row y-1 run at the same time on
// double-buffered operand tables, so the VALU and matrix pipes of a SIMD
// overlap; there is one barrier per input row.
//
// Convolution waves share one code path (their planes are data).  A lane
// owns one output column: it keeps the last 2h+1 row-filtered values of each
// of its planes in registers (a window that advances one row per step and is
// re-based every U steps), so the column pass reads no LDS.  Both passes use
// the symmetry of the filters, f(-u) = (-1)^i f(u): the taps at +-u are
// added (even i) or subtracted (odd i) first, which halves the coefficients
// a filter needs.
//
// The operand tables are k-major (c[k][p]) so that a lane's operands of
// four consecutive MFMA steps are one 16-byte LDS read; the per-row sums
// take the pixels in a different order than fit_wave, otherwise the
// moments, products and FP64 flushes are those of fit_wave.
#pragma once
#include <type_traits>
#include "fit_accum.h"

namespace argus_fit {

constexpr int U8 = 4;       // steps between re-basings of the column windows

// Steps (and barriers) of a strip: n row steps padded to whole blocks of U8.
__device__ __forceinline__ int fit8_steps(int n) { return (n + U8 - 1) / U8 * U8; }

// TS (the BF16x3 form): the fixed-up basis rows c' and their bf16 hi/lo
// split are built once per row by the convolution waves, one step after the
// row's convolution (every MFMA wave used to form and split all 2048 of them
// itself); with copies of the row's weights they feed the MFMA waves one step
// later.  The values and their split are those the MFMA waves computed.
template <int D, int HH, bool TS = false>
struct FitLds8 {
    static constexpr int K = 2 * HH + 1;
    static constexpr int IN = SW + 2 * HH;               // input row length
    static constexpr int INP = (IN + 3) & ~3;
    static constexpr int CKM = SW + 4;                   // k-major row stride of c
    static constexpr int CKB = SW + 8;                   // row stride of the bf16 tables (16-byte rows)
    // TS block per buffer: c' [32][CKM] f32, hi and lo [32][CKB] bf16, copies
    // of w xt^a [NA][SW] and w s xt^e [NRA][SW]
    static constexpr int TSB = 32 * CKM + 32 * CKB + (FitShape<D>::NA + FitShape<D>::NRA) * SW;
    float *inrow, *cvec0, *wx0, *wsx0;
    double *wxd0, *wsxd0;
    float *ts0 = nullptr;
    uint64_t *mbits;                                     // [2][2] flagged input pixels
    __device__ float *tsc(int b) const { return ts0 + b * TSB; }
    __device__ __bf16 *tsh(int b) const { return (__bf16 *)(tsc(b) + 32 * CKM); }
    __device__ __bf16 *tsl(int b) const { return tsh(b) + 32 * CKB; }
    __device__ float *tswx(int b) const { return tsc(b) + 32 * CKM + 32 * CKB; }
    __device__ float *tswsx(int b) const { return tswx(b) + FitShape<D>::NA * SW; }
    // buffer b (0/1) of each double-buffered table (no pointer arrays: a
    // runtime index into one would place it in scratch)
    __device__ float *cvec(int b) const { return cvec0 + b * (32 * CKM); }
    __device__ float *wx(int b) const { return wx0 + b * (FitShape<D>::NA * SW); }
    __device__ float *wsx(int b) const { return wsx0 + b * (FitShape<D>::NRA * SW); }
    __device__ double *wxd(int b) const { return wxd0 + b * (FitShape<D>::NA * SW); }
    __device__ double *wsxd(int b) const { return wsxd0 + b * (FitShape<D>::NRA * SW); }
    __host__ __device__ static size_t bytes(int nwm) {
        using S = FitShape<D>;
        size_t w = 2 * INP + 2 * 32 * CKM + 2 * (S::NA + S::NRA) * SW + (TS ? 2 * TSB : 0);
        size_t b = w * 4 + (size_t)2 * (S::NA + S::NRA) * SW * 8 + 4 * 8;
        size_t rhs = (size_t)2 * nwm * S::NR * 32 * 8;   // end-of-kernel reuse
        return (b > rhs ? b : rhs) + 64;
    }
    __device__ FitLds8(float *lds) {
        using S = FitShape<D>;
        inrow = lds;                                    // [2][INP] double-buffered input row
        cvec0 = inrow + 2 * INP;                        // [2][32][CKM] k-major
        wx0 = cvec0 + 2 * 32 * CKM;                     // [2][NA][SW]
        wsx0 = wx0 + 2 * S::NA * SW;                    // [2][NRA][SW]
        // every region above is a multiple of 16 bytes long (INP, SW, CKM are
        // multiples of 4): no integer round trip, which would turn the LDS
        // pointers into generic ones
        wxd0 = (double *)(wsx0 + 2 * S::NRA * SW);
        wsxd0 = wxd0 + 2 * S::NA * SW;
        mbits = (uint64_t *)(wsxd0 + 2 * S::NRA * SW);
        if (TS) ts0 = (float *)(mbits + 4);             // [2][TSB] (TSB is a multiple of 4)
    }
};

// Steps of a strip: the input rows plus the rows the pipeline drains (the
// moments of output row y run one step after its convolution, TS's two).
template <bool TS>
__device__ __forceinline__ int fit8_strip_steps(int rows) { return fit8_steps(rows + (TS ? 2 : 1)); }

// Convolution wave cw (wave-uniform) of the NWC convolution waves, with up
// to NP planes (from plist8 for 8 waves, plist for 4).  Wave 0 (W0) also
// stages the fit-set weights (with 8 waves it takes one plane, so that its
// registers fit the same budget); it returns the number of fit pixels it
// counted, the others return 0.
template <int D, int HH, int PREC, int NWC, int NP, bool W0>
__device__ int fit_conv8(const FitArgs &a, float *lds, int sx_begin, int sx_end, int ry0,
                         int ry1, bool active, int cw) {
    using S = FitShape<D>;
    constexpr bool TS = PREC == ARGUS_BF16X3;
    using L = FitLds8<D, HH, TS>;
    constexpr int K = L::K;
    constexpr int NR_ = K - 1 + U8;                      // window registers per plane
    const int tid = threadIdx.x, lane = tid & 63;
    L l(lds);
    int count = 0;

    // this wave's planes and their first basis function / basis count
    int pl[NP], k0[NP], nk[NP];
    float rc[NP][HH + 1];                                // row filter, taps 0..h
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        pl[j] = NWC == 8 ? a.plist8[cw][j] : a.plist[cw][j];
        k0[j] = 0;
        nk[j] = 0;
        if (pl[j] >= 0) {
            for (int k = 0; k < a.nb; ++k)
                if (a.tab->kpl[k] == pl[j]) {
                    if (nk[j] == 0) k0[j] = k;
                    ++nk[j];
                }
        }
        k0[j] = __builtin_amdgcn_readfirstlane(k0[j]);
        nk[j] = __builtin_amdgcn_readfirstlane(nk[j]);
        const int p = pl[j] >= 0 ? pl[j] : 0;
#pragma unroll
        for (int v = 0; v <= HH; ++v) {
            rc[j][v] = uload(&a.tab->rowf[p][HH + v]);
        }
    }
    // parity of each plane's row filter in x (odd filters vanish at u = 0)
    bool odd[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j)
        odd[j] = __builtin_amdgcn_readfirstlane(pl[j] >= 0 ? a.tab->ipow[pl[j]] & 1 : 0) != 0;

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
        // Waves 0 and 1 hold the IN input pixels.
        float pr = 0.f;
        uint8_t pm = 0;
        float p_s = 0.f, p_sv = 0.f, p_rv = 0.f;
        uint8_t p_sm = 1;
        bool pok = false;
        const bool stager = cw * 64 + lane < L::IN;
        const int Xin = sx0 - HH + cw * 64 + lane;
        const bool in_x = stager && Xin >= 0 && Xin < a.W;
        const int Xc = in_x ? Xin : (Xin < 0 ? 0 : a.W - 1);
        auto fetch_in = [&](int yy) {
            if (cw < 2 && stager) {
                pr = a.ref[(int64_t)yy * P + Xc];
                pm = a.rmask[(int64_t)yy * P + Xc];
            }
        };
        const bool lane_ok = sx0 + lane < sx1;
        const int64_t xw = lane_ok ? sx0 + lane : sx0;
        auto fetch_w = [&](int y) {
            pok = lane_ok && y >= ry0 && y < ry1;
            const int yc = y < ry1 ? y : ry1 - 1;
            const int64_t o = (int64_t)yc * P + xw;
            p_s = a.sci[o];
            p_sv = a.svar[o];
            p_rv = a.rvar[o];
            p_sm = a.smask[o];
        };
        auto stage = [&](int b) {
            if (cw < 2) {
                const bool f = stager && in_x && pm != 0;
                const uint64_t bits = __ballot(f);
                if (stager) l.inrow[b * L::INP + cw * 64 + lane] = in_x ? pr : 0.f;
                if (lane == 0) l.mbits[2 * b + cw] = bits;
            }
        };
        uint32_t hist = 0;                 // bit j: input row yy-j has a flagged pixel in reach
        bool pend = false;                 // TS: the previous step wrote an output row's c
        const int ystart = ry0 - HH;
        const int yend = active ? ry1 + HH : ystart;
        if (active) {
            fetch_in(ystart);
            stage(ystart & 1);
            if (ystart + 1 < yend) fetch_in(ystart + 1);
            if (W0) fetch_w(ry0);
        }
        __syncthreads();
        float rw[NP][NR_];                 // column windows: rw[j][u .. u+K-1] at sub-step u
#pragma unroll
        for (int j = 0; j < NP; ++j)
#pragma unroll
            for (int i = 0; i < NR_; ++i) rw[j][i] = 0.f;

        // One step: input row yy (sub-step u of a block of U8).  Steps at and
        // after yend only keep the barrier count; their row pass runs on stale
        // LDS data (in bounds) into window slots that no output uses, which
        // keeps the window registers free of conditional updates.
        auto step = [&](auto uc, int yy) {
            constexpr int u = decltype(uc)::value;
            // steps start at an even row (ys0), so the buffer parity is the
            // sub-step's: every table address is a constant offset
            constexpr int buf = u & 1;
            const bool live = yy >= ystart && yy < yend;
            if (live) {
                if (yy + 1 < yend) stage(buf ^ 1);
                if (yy + 2 < yend) fetch_in(yy + 2);
            }
            const float w_s = p_s, w_sv = p_sv, w_rv = p_rv;
            const uint8_t w_sm = pok ? p_sm : 1;
            const bool outrow = live && yy >= ry0 + HH;
            if (W0 && outrow) fetch_w(yy + 1 - HH);
            {
                // row pass: taps +-v of the input row paired
                {
                    const float *ir = l.inrow + buf * L::INP + lane + HH;
                    float sp[HH + 1], sm[HH + 1];
                    const float c = ir[0];
#pragma unroll
                    for (int v = 1; v <= HH; ++v) {
                        const float lo = ir[-v], hi = ir[v];
                        sp[v] = lo + hi;
                        sm[v] = lo - hi;
                    }
#pragma unroll
                    for (int j = 0; j < NP; ++j) {
                        float acc;
                        if (odd[j]) {
                            acc = rc[j][1] * sm[1];
#pragma unroll
                            for (int v = 2; v <= HH; ++v) acc += rc[j][v] * sm[v];
                        } else {
                            acc = rc[j][0] * c;
#pragma unroll
                            for (int v = 1; v <= HH; ++v) acc += rc[j][v] * sp[v];
                        }
                        rw[j][K - 1 + u] = acc;
                    }
                }
                if (W0 && live) {
                    // flagged reference pixel within +-h of this column
                    const uint64_t b0 = l.mbits[2 * buf], b1 = l.mbits[2 * buf + 1];
                    const uint64_t lo = (b0 >> lane) | ((b1 << (63 - lane)) << 1);
                    const bool m = (lo & ((1ull << K) - 1ull)) != 0;
                    hist = (hist << 1) | (m ? 1u : 0u);
                }
                if (outrow) {
                    // column pass: rows y-h..y+h are rw[j][u .. u+2h]
                    float *cv = l.cvec(buf);
#pragma unroll
                    for (int j = 0; j < NP; ++j) {
                        if (nk[j] > 0) {
                            // even column powers on the paired sums, then odd
                            // ones on the paired differences
                            float e[HH + 1];
                            e[0] = rw[j][u + HH];
#pragma unroll
                            for (int v = 1; v <= HH; ++v) e[v] = rw[j][u + HH - v] + rw[j][u + HH + v];
#pragma unroll
                            for (int q = 0; q < 7; q += 2) {
                                if (q < nk[j]) {
                                    const float *f = &a.tab->colf[k0[j] + q][HH];
                                    float acc = uload(f) * e[0];
#pragma unroll
                                    for (int v = 1; v <= HH; ++v) acc += uload(f + v) * e[v];
                                    cv[(k0[j] + q) * L::CKM + lane] = acc;
                                }
                            }
                            if (nk[j] > 1) {
#pragma unroll
                                for (int v = 1; v <= HH; ++v) e[v] = rw[j][u + HH - v] - rw[j][u + HH + v];
#pragma unroll
                                for (int q = 1; q < 7; q += 2) {
                                    if (q < nk[j]) {
                                        const float *f = &a.tab->colf[k0[j] + q][HH];
                                        float acc = uload(f + 1) * e[1];
#pragma unroll
                                        for (int v = 2; v <= HH; ++v) acc += uload(f + v) * e[v];
                                        cv[(k0[j] + q) * L::CKM + lane] = acc;
                                    }
                                }
                            }
                        }
                    }
                    if (W0) {
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
            if constexpr (TS) {
                // split tables of the previous step's output row: this wave's
                // four basis rows k, fixed up (c'_k = c_k + gam_k c_0; the
                // background row is 1, rows past it stay zero), and their
                // bf16 hi/lo parts; the last wave copies the row's weights
                if (pend) {
                    const int pb = buf ^ 1;
                    const float *cv = l.cvec(pb);
                    const float c0v = cv[lane];
                    float *tc = l.tsc(buf);
                    __bf16 *th = l.tsh(buf), *tl = l.tsl(buf);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int k = cw * 4 + q;
                        if (k <= a.nb) {
                            const float c = k < a.nb ? cv[k * L::CKM + lane] + uload(&a.tab->gam[k]) * c0v
                                                     : 1.f;
                            const __bf16 h = (__bf16)c;
                            tc[k * L::CKM + lane] = c;
                            th[k * L::CKB + lane] = h;
                            tl[k * L::CKB + lane] = (__bf16)(c - (float)h);
                        }
                    }
                    if (cw == NWC - 1) {
#pragma unroll
                        for (int e = 0; e < S::NA; ++e) l.tswx(buf)[e * SW + lane] = l.wx(pb)[e * SW + lane];
#pragma unroll
                        for (int e = 0; e < S::NRA; ++e) l.tswsx(buf)[e * SW + lane] = l.wsx(pb)[e * SW + lane];
                    }
                }
                pend = outrow;
            }
            __syncthreads();
        };
        // extra steps drain the last output row into the moments; the step
        // count is padded to whole blocks (the MFMA waves count alike)
        // (an odd first row gets one leading step that only keeps the count)
        const int ys0 = ystart & ~1;
        const int ylast = ys0 + fit8_strip_steps<TS>(yend - ys0) - 1;
        for (int yy = ys0; yy <= ylast; yy += U8) {
            step(std::integral_constant<int, 0>{}, yy);
            step(std::integral_constant<int, 1>{}, yy + 1);
            step(std::integral_constant<int, 2>{}, yy + 2);
            step(std::integral_constant<int, 3>{}, yy + 3);
            // re-base the windows: the newest K-1 rows move to the front
#pragma unroll
            for (int j = 0; j < NP; ++j)
#pragma unroll
                for (int i = 0; i < K - 1; ++i) rw[j][i] = rw[j][i + U8];
        }
    }
    return count;
}

// TS: the moments of one row into acc from the split tables (tc: c', th/tl:
// its hi/lo parts, wx: w xt^a).  A lane takes 8 pixels per 32-pixel step: the
// A operands are read split; B = w xt^a c'_l is formed and split here (it
// differs per task); the products hi*hi, hi*lo, lo*hi in that order.
template <int MW, int STR, int NTW, int CKM, int CKB>
__device__ __forceinline__ void row_ts_acc(const float *tc, const __bf16 *th, const __bf16 *tl,
                                           const float *wx, int lane,
                                           floatx4 (&acc)[NTW > 0 ? NTW : 1]) {
    if constexpr (NTW > 0) {
        const int col = lane & 15, pk = lane >> 4;
#pragma unroll
        for (int j = 0; j < NTW; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < SW / 32; ++s) {
            const int p0 = 32 * s + 8 * pk;
            const bf16x8 h0 = *(const bf16x8 *)(th + col * CKB + p0);
            const bf16x8 l0 = *(const bf16x8 *)(tl + col * CKB + p0);
            const bf16x8 h1 = *(const bf16x8 *)(th + (16 + col) * CKB + p0);
            const bf16x8 l1 = *(const bf16x8 *)(tl + (16 + col) * CKB + p0);
            float c0[8], c1[8];
            {
                const float4 a0 = *(const float4 *)(tc + col * CKM + p0);
                const float4 a1 = *(const float4 *)(tc + col * CKM + p0 + 4);
                const float4 b0 = *(const float4 *)(tc + (16 + col) * CKM + p0);
                const float4 b1 = *(const float4 *)(tc + (16 + col) * CKM + p0 + 4);
                c0[0] = a0.x; c0[1] = a0.y; c0[2] = a0.z; c0[3] = a0.w;
                c0[4] = a1.x; c0[5] = a1.y; c0[6] = a1.z; c0[7] = a1.w;
                c1[0] = b0.x; c1[1] = b0.y; c1[2] = b0.z; c1[3] = b0.w;
                c1[4] = b1.x; c1[5] = b1.y; c1[6] = b1.z; c1[7] = b1.w;
            }
#pragma unroll
            for (int j = 0; j < NTW; ++j) {
                const int t = MW + STR * j;
                const int a = t / 3, bp = t % 3;
                const float4 w0 = *(const float4 *)(wx + a * SW + p0);
                const float4 w1 = *(const float4 *)(wx + a * SW + p0 + 4);
                const float wv[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
                bf16x8 bh, bl;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float B = wv[e] * ((bp == 0) ? c0[e] : c1[e]);
                    const __bf16 bb = (__bf16)B;
                    bh[e] = bb;
                    bl[e] = (__bf16)(B - (float)bb);
                }
                const bf16x8 ah = (bp == 2) ? h1 : h0;
                const bf16x8 al = (bp == 2) ? l1 : l0;
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[j], 0, 0, 0);
            }
        }
    }
}

// MFMA wave W (NWC <= W < NWC + NWM) of the workgroup: the moments of the
// previous output row from the tables the convolution waves wrote, and the
// right-hand-side pieces of its pixels.
template <int D, int HH, int W, int PREC, int NWC, int NWM>
__device__ void fit_mfma8(const FitArgs &a, float *lds, int sx_begin, int sx_end, int ry0,
                          int ry1, bool active, double *part) {
    using S = FitShape<D>;
    constexpr bool TS = PREC == ARGUS_BF16X3;
    using L = FitLds8<D, HH, TS>;
    constexpr int MW = W - NWC;
    constexpr int PXW = SW / NWM, PXH = PXW / 2;         // rhs pixels per wave and half-wave
    const int tid = threadIdx.x, lane = tid & 63;
    L l(lds);
    double *rhsbuf = (double *)lds;

    using G = WaveGram<D, MW, PREC, NWM>;
    G gram;
    double RF[S::NR];
    gram.zero();
    // Of the two MFMA waves on a SIMD (MW and MW + NWM/2), the second flushes
    // a row's moments at the start of the next step, before its right-hand
    // side and MFMAs: its VALU work then overlaps its partner's MFMAs (and
    // the other way round) instead of both waves using the matrix pipe and
    // the VALU at the same times.
    constexpr bool DEFER = NWM == 8 && MW >= NWM / 2;
    typename G::Acc acc[G::NTW > 0 ? G::NTW : 1];
    bool have = false;
    int yprev = 0;
    auto ypowers = [&](int yv, double *ypw) {
        const double yt = (double)yv * a.sy - (a.sy != 0.0 ? 1.0 : 0.0);
        double yp = 1.0;
#pragma unroll
        for (int b = 0; b <= 2 * D; ++b) { ypw[b] = yp; yp *= yt; }
    };
#pragma unroll
    for (int i = 0; i < S::NR; ++i) RF[i] = 0.0;
    const float g0 = (lane & 15) < a.nb ? a.tab->gam[lane & 15] : 0.f;
    const float g1 = 16 + (lane & 15) < a.nb ? a.tab->gam[16 + (lane & 15)] : 0.f;
    const float gk = (lane & 31) < a.nb ? a.tab->gam[lane & 31] : 0.f;  // rhs fix-up
    const int nstrips = active ? (sx_end - sx_begin + SW - 1) / SW : 1;
    for (int strip = 0; strip < nstrips; ++strip) {
        const int ystart = ry0 - HH;
        const int yend = active ? ry1 + HH : ystart;
        const int ys0 = ystart & ~1;                 // the convolution waves' first step
        const int ylast = ys0 + fit8_strip_steps<TS>(yend - ys0) - 1;
        __syncthreads();
        for (int yy = ys0; yy <= ylast; ++yy) {
            const int buf = yy & 1;
            if constexpr (TS) {
                // moments of output row y = yy - 2 - h: its c was convolved two
                // steps ago and its split tables built in the previous step
                const int y = yy - 2 - HH;
                if (yy - 2 >= ry0 + HH && yy - 2 < yend) {
                    const int pb = buf ^ 1;
                    double ypw[2 * D + 1];
                    if constexpr (DEFER) {
                        if (have) {
                            ypowers(yprev, ypw);
                            gram.flush(acc, ypw);
                        }
                    }
                    ypowers(y, ypw);
                    if constexpr (!DEFER) {
                        row_ts_acc<MW, NWM, G::NTW, L::CKM, L::CKB>(l.tsc(pb), l.tsh(pb), l.tsl(pb),
                                                                     l.tswx(pb), lane, acc);
                        gram.flush(acc, ypw);
                    }
                    // rhs pieces of this half-wave's pixels: w s xt^e c'_k
                    const int k = lane & 31, half = lane >> 5;
                    float ra[S::NRA];
#pragma unroll
                    for (int e = 0; e < S::NRA; ++e) ra[e] = 0.f;
#pragma unroll
                    for (int i = 0; i < PXH; ++i) {
                        const int px = MW * PXW + half * PXH + i;
                        const float c = l.tsc(pb)[k * L::CKM + px];
#pragma unroll
                        for (int e = 0; e < S::NRA; ++e) ra[e] += l.tswsx(pb)[e * SW + px] * c;
                    }
#pragma unroll
                    for (int e = 0; e < S::NRA; ++e)
#pragma unroll
                        for (int b = 0; b <= D; ++b)
                            if (e + b <= D) RF[qidx(e, b, D)] += ypw[b] * (double)ra[e];
                    if constexpr (DEFER) {
                        row_ts_acc<MW, NWM, G::NTW, L::CKM, L::CKB>(l.tsc(pb), l.tsh(pb), l.tsl(pb),
                                                                     l.tswx(pb), lane, acc);
                        have = true;
                        yprev = y;
                    }
                }
                __syncthreads();
                continue;
            }
            // moments of output row y = yy - 1 - h, written during the previous step
            const int y = yy - 1 - HH;
            if (yy - 1 >= ry0 + HH && yy - 1 < yend) {
                const int pb = buf ^ 1;
                double ypw[2 * D + 1];
                if constexpr (DEFER) {
                    if (have) {
                        ypowers(yprev, ypw);
                        gram.flush(acc, ypw);
                    }
                }
                ypowers(y, ypw);
                if constexpr (!DEFER) gram.row_km(l.cvec(pb), l.wx(pb), l.wxd(pb), ypw, lane, g0, g1);
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
                if constexpr (DEFER) {
                    gram.row_km_acc(l.cvec(pb), l.wx(pb), l.wxd(pb), lane, g0, g1, acc);
                    have = true;
                    yprev = y;
                }
            }
            __syncthreads();
        }
    }
    if constexpr (DEFER) {
        if (have) {
            double ypw[2 * D + 1];
            ypowers(yprev, ypw);
            gram.flush(acc, ypw);
        }
    }
    // partials: moments, rhs pieces through LDS (summed by the whole workgroup)
    gram.store(part, lane);
    const int k = lane & 31, half = lane >> 5;
#pragma unroll
    for (int i = 0; i < S::NR; ++i) rhsbuf[((MW * 2 + half) * S::NR + i) * 32 + k] = RF[i];
}

template <int D, int HH, int PREC, int NWC, int NWM, int W>
__device__ __forceinline__ void fit_dispatch8(int w, const FitArgs &a, float *lds, int sx0, int sx1,
                                              int ry0, int ry1, bool active, double *part) {
    if constexpr (W < NWC + NWM) {
        if (w == W)
            fit_mfma8<D, HH, W, PREC, NWC, NWM>(a, lds, sx0, sx1, ry0, ry1, active, part);
        else
            fit_dispatch8<D, HH, PREC, NWC, NWM, W + 1>(w, a, lds, sx0, sx1, ry0, ry1, active, part);
    }
}

template <int D, int HH, int PREC, int NWC, int NWM>
__global__ __launch_bounds__(64 * (NWC + NWM)) void fit_accum8_kernel(FitArgs a) {
    extern __shared__ __align__(16) float lds[];
    using S = FitShape<D>;
    constexpr int NTH = 64 * (NWC + NWM);
    // planes per convolution wave: 8 waves take 1 (wave 0) or 2, 4 waves up to 4
    constexpr int NP0 = NWC == 8 ? 1 : 4, NP = NWC == 8 ? 2 : 4;
    const int tid = threadIdx.x;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
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
    // constant tail of c: 1 at index nb (background), zeros after, both
    // buffers; with split tables (BF16x3) their rows past nb are zero too
    constexpr bool TS = PREC == ARGUS_BF16X3;
    using LT = FitLds8<D, HH, TS>;
    LT L(lds);
    for (int i = tid; i < 2 * 32 * LT::CKM; i += NTH) {
        const int k = (i / LT::CKM) % 32;
        if (k >= a.nb) L.cvec0[i] = (k == a.nb) ? 1.f : 0.f;
    }
    if constexpr (TS) {
        for (int i = tid; i < 2 * 32 * LT::CKM; i += NTH) {
            const int b = i / (32 * LT::CKM), k = (i / LT::CKM) % 32;
            if (k > a.nb) L.tsc(b)[i % (32 * LT::CKM)] = 0.f;
        }
        for (int i = tid; i < 2 * 32 * LT::CKB; i += NTH) {
            const int b = i / (32 * LT::CKB), k = (i / LT::CKB) % 32, r = i % (32 * LT::CKB);
            if (k > a.nb) {
                L.tsh(b)[r] = (__bf16)0.f;
                L.tsl(b)[r] = (__bf16)0.f;
            }
        }
    }
    int count = 0;
    if (w == 0)
        count = fit_conv8<D, HH, PREC, NWC, NP0, true>(a, lds, sx0, sx1, ry0, ry1, active, 0);
    else if (w < NWC)
        fit_conv8<D, HH, PREC, NWC, NP, false>(a, lds, sx0, sx1, ry0, ry1, active, w);
    else
        fit_dispatch8<D, HH, PREC, NWC, NWM, NWC>(w, a, lds, sx0, sx1, ry0, ry1, active, part);
    if (w == 0) {
        const int lane = tid & 63;
        double c = (double)count;
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
        if (lane == 0) part[(size_t)S::NQ * 768 + S::NR * 32] = c;
    }
    __syncthreads();
    const double *rhsbuf = (const double *)lds;
    for (int it = tid; it < S::NR * 32; it += NTH) {
        double acc = 0.0;
        for (int q = 0; q < 2 * NWM; ++q) acc += rhsbuf[q * S::NR * 32 + it];
        part[(size_t)S::NQ * 768 + it] = acc;
    }
}

// Launch fit_accum8_kernel<D, h, PREC, NWC, NWM> with its dynamic LDS size:
// FP32 and BF16x3 run 8 convolution + 8 MFMA waves (two tasks each, so every
// wave fits in 128 registers and each SIMD holds four waves); FP64, whose
// 64-bit MFMA operands and accumulators do not fit that budget, runs 4 + 4
// with four tasks per MFMA wave.
template <int PREC>
int fit_accum8_launch(argus_ctx *ctx, const FitArgs &fa, int D, dim3 grid) {
    constexpr int NWM = PREC == ARGUS_FP64 ? 4 : 8;
    constexpr int NWC = PREC == ARGUS_FP64 ? 4 : 8;
    hipError_t err = hipSuccess;
    bool ok = false;
#define ARGUS_FH(DD, HH)                                                                   \
    if (D == DD && fa.h == HH) {                                                           \
        size_t lds = FitLds8<DD, HH, PREC == ARGUS_BF16X3>::bytes(NWM);                    \
        err = hipFuncSetAttribute((const void *)fit_accum8_kernel<DD, HH, PREC, NWC, NWM>, \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        if (err == hipSuccess)                                                             \
            hipLaunchKernelGGL((fit_accum8_kernel<DD, HH, PREC, NWC, NWM>), grid,          \
                               dim3(64 * (NWC + NWM)), lds, ctx->stream, fa);              \
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
