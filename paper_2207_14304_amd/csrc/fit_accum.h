// Fused basis convolution + normal-equation moment accumulation (shared by
// the per-precision translation units k_fit_fp32/fp64/bf16.hip).
//
// Every entry of A = sum w X X^T is a moment G_ab[k][l] = sum_p w xt^a yt^b
// c_k c_l of the 32-vector c = (C_0..C_{nb-1}, 1, 0...) with a+b <= 2D, and
// b needs R_ab[k] = sum w xt^a yt^b c_k S with a+b <= D.  Along one image row
// yt is constant, so a workgroup accumulates the 2D+1 xt-moments of each row
// on MFMA (three 16x16 blocks of the symmetric 32x32 moment per power) and
// adds yt^b times them into FP64 running sums.
//
// Precisions of the per-row products and sums:
//   ARGUS_FP32   FP32 operands, v_mfma_f32_16x16x4f32 over 64 pixels;
//   ARGUS_FP64   FP64 operands, v_mfma_f64_16x16x4f64 (FP64 products and sums);
//   ARGUS_BF16X3 x = hi + lo with hi, lo bf16 (round to nearest even), and
//                A B ~ Ahi Bhi + Ahi Blo + Alo Bhi on v_mfma_f32_16x16x32_bf16
//                with FP32 accumulation (Henry, Tang & Heinecke 2019).
#pragma once
#include <type_traits>

#include "internal.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace argus_fit {

constexpr int SW = 64;        // output columns per workgroup strip
constexpr int CST = 33;       // LDS row stride of the 32-vector c (bank spread)
constexpr int NTHR = 256;

// ---------------------------------------------------------------------------
struct FitArgs {
    const float *ref, *rvar, *sci, *svar;
    const uint8_t *rmask, *smask;
    const BasisTables *tab;
    double *partials;
    int64_t pitch;
    int W, H, h, nb, nplanes;
    int RX, RY;                // regions (1x1 for GLOBAL, tiles for PER_TILE)
    int spt, rchunks;          // strips per region, row chunks per region
    int stride;                // doubles per partial
    double sx, sy;             // 2/(W-1), 2/(H-1) (0 for a 1-pixel axis)
    int8_t plist[4][4];        // row-filter planes of each wave (-1: none)
    int8_t plist8[8][2];       // the same for 8 convolution waves
};

__device__ __forceinline__ int qidx(int a, int b, int Dm) {   // a+b <= Dm, a outer
    return a * (Dm + 1) - a * (a - 1) / 2 + b;
}

template <int D>
struct FitShape {
    static constexpr int NA = 2 * D + 1;                       // xt powers in the Gram
    static constexpr int NQ = (2 * D + 1) * (2 * D + 2) / 2;   // Gram moments
    static constexpr int NRA = D + 1;                          // xt powers in the rhs
    static constexpr int NR = (D + 1) * (D + 2) / 2;           // rhs moments
    static constexpr int NT = 3 * NA;                          // (a, block pair) tasks
};

// Per-wave MFMA work on one 64-pixel row: tasks t = WAVE, WAVE+4, ... with
// a = t / 3 and block pair bp = t % 3 in {(0,0), (0,1), (1,1)}.
template <int D, int WAVE, int PREC, int STR = 4>
struct WaveGram {
    // tasks t = WAVE, WAVE + STR, ... of the 3 (2D+1) (power, block pair) tasks
    static constexpr int NT = FitShape<D>::NT;
    static constexpr int NTW = (NT - WAVE + STR - 1) / STR;
    static constexpr int NB = 2 * D + 1;
    double F[NTW > 0 ? NTW : 1][NB][4];

    __device__ void zero() {
#pragma unroll
        for (int j = 0; j < (NTW > 0 ? NTW : 1); ++j)
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) F[j][b][r] = 0.0;
    }

    template <typename V>
    __device__ void flush(const V (&acc)[NTW > 0 ? NTW : 1], const double *ypw) {
#pragma unroll
        for (int j = 0; j < NTW; ++j) {
            const int a = (WAVE + STR * j) / 3;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (b <= 2 * D - a) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) F[j][b][r] += ypw[b] * (double)acc[j][r];
                }
            }
        }
    }

    // c'_k = c_k + gam_k c_0 is applied to the operands as they are loaded.
    __device__ void row(const float *cvec, const float *wx, const double *wxd, const double *ypw,
                        int lane, float g0, float g1) {
        if constexpr (NTW > 0) {
            const int col = lane & 15, pk = lane >> 4;
            if constexpr (PREC == ARGUS_FP32) {
                floatx4 acc[NTW];
#pragma unroll
                for (int j = 0; j < NTW; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
                // operands of step s+1 are loaded while the MFMAs of step s run
                float nz, n0, n1, nw[NTW];
                auto load = [&](int s) {
                    const int p = 4 * s + pk;
                    nz = cvec[p * CST];
                    n0 = cvec[p * CST + col];
                    n1 = cvec[p * CST + 16 + col];
#pragma unroll
                    for (int j = 0; j < NTW; ++j) nw[j] = wx[((WAVE + STR * j) / 3) * SW + p];
                };
                load(0);
#pragma unroll
                for (int s = 0; s < SW / 4; ++s) {
                    const float cz = nz, r0 = n0, r1 = n1;
                    float wa[NTW];
#pragma unroll
                    for (int j = 0; j < NTW; ++j) wa[j] = nw[j];
                    if (s + 1 < SW / 4) load(s + 1);
                    const float c0 = r0 + g0 * cz;
                    const float c1 = r1 + g1 * cz;
#pragma unroll
                    for (int j = 0; j < NTW; ++j) {
                        const int t = WAVE + STR * j;
                        const int bp = t % 3;
                        const float A = (bp == 2) ? c1 : c0;
                        const float B = wa[j] * ((bp == 0) ? c0 : c1);
                        acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A, B, acc[j], 0, 0, 0);
                    }
                }
                flush(acc, ypw);
            } else if constexpr (PREC == ARGUS_FP64) {
                doublex4 acc[NTW];
#pragma unroll
                for (int j = 0; j < NTW; ++j) acc[j] = doublex4{0.0, 0.0, 0.0, 0.0};
                float nz, n0, n1;
                double nw[NTW];
                auto load = [&](int s) {
                    const int p = 4 * s + pk;
                    nz = cvec[p * CST];
                    n0 = cvec[p * CST + col];
                    n1 = cvec[p * CST + 16 + col];
#pragma unroll
                    for (int j = 0; j < NTW; ++j) nw[j] = wxd[((WAVE + STR * j) / 3) * SW + p];
                };
                load(0);
#pragma unroll
                for (int s = 0; s < SW / 4; ++s) {
                    const double cz = (double)nz;
                    const double c0 = (double)n0 + (double)g0 * cz;
                    const double c1 = (double)n1 + (double)g1 * cz;
                    double wa[NTW];
#pragma unroll
                    for (int j = 0; j < NTW; ++j) wa[j] = nw[j];
                    if (s + 1 < SW / 4) load(s + 1);
#pragma unroll
                    for (int j = 0; j < NTW; ++j) {
                        const int t = WAVE + STR * j;
                        const int bp = t % 3;
                        const double A = (bp == 2) ? c1 : c0;
                        const double B = wa[j] * ((bp == 0) ? c0 : c1);
                        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(A, B, acc[j], 0, 0, 0);
                    }
                }
                flush(acc, ypw);
            } else {
                floatx4 acc[NTW];
#pragma unroll
                for (int j = 0; j < NTW; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < SW / 32; ++s) {
                    // this lane's 8 pixels of the 32-pixel step
                    float c0[8], c1[8];
                    bf16x8 h0, l0, h1, l1;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int p = 32 * s + 8 * pk + e;
                        const float cz = cvec[p * CST];
                        c0[e] = cvec[p * CST + col] + g0 * cz;
                        c1[e] = cvec[p * CST + 16 + col] + g1 * cz;
                        const __bf16 a0 = (__bf16)c0[e], a1 = (__bf16)c1[e];
                        h0[e] = a0;
                        l0[e] = (__bf16)(c0[e] - (float)a0);
                        h1[e] = a1;
                        l1[e] = (__bf16)(c1[e] - (float)a1);
                    }
#pragma unroll
                    for (int j = 0; j < NTW; ++j) {
                        const int t = WAVE + STR * j;
                        const int a = t / 3, bp = t % 3;
                        bf16x8 bh, bl;
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const int p = 32 * s + 8 * pk + e;
                            const float B = wx[a * SW + p] * ((bp == 0) ? c0[e] : c1[e]);
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
                flush(acc, ypw);
            }
        }
    }

    // The same row on k-major operand tables: c[k][p] with row stride CKM
    // and w xt^a [a][p]; at step s the four lane groups pk take the pixels
    // p = 16 pk + s (FP32, FP64) or p = 32 s + 8 pk + e (BF16X3), so a lane's
    // operands of consecutive steps are contiguous and load 16 bytes at once.
    static constexpr int CKM = SW + 4;
    // Accumulator of one task: 4 FP32 (FP64 for ARGUS_FP64) values per lane.
    using Acc = typename std::conditional<PREC == ARGUS_FP64, doublex4, floatx4>::type;

    // The moments of one row into acc (not yet flushed into the FP64 sums).
    __device__ void row_km_acc(const float *cvec, const float *wx, const double *wxd, int lane,
                               float g0, float g1, Acc (&acc)[NTW > 0 ? NTW : 1]) {
        if constexpr (NTW > 0) {
            const int col = lane & 15, pk = lane >> 4;
            if constexpr (PREC == ARGUS_FP32 || PREC == ARGUS_FP64) {
                using T = typename std::conditional<PREC == ARGUS_FP32, float, double>::type;
                using TV = typename std::conditional<PREC == ARGUS_FP32, floatx4, doublex4>::type;
                const float *pa = cvec + col * CKM + 16 * pk;
                const float *pb = cvec + (16 + col) * CKM + 16 * pk;
                const float *pz = cvec + 16 * pk;
#pragma unroll
                for (int j = 0; j < NTW; ++j) acc[j] = TV{0, 0, 0, 0};
                // the operands of 4 steps are loaded while the 4 steps before run
                float4 na, nb, nz;
                T nw[NTW][4];
                // (FP64: the weights are read in their own group, as two
                // groups of FP64 weights do not fit the register budget)
                auto load = [&](int u) {
                    na = *(const float4 *)(pa + 4 * u);
                    nb = *(const float4 *)(pb + 4 * u);
                    nz = *(const float4 *)(pz + 4 * u);
                    if constexpr (PREC == ARGUS_FP32) {
#pragma unroll
                        for (int j = 0; j < NTW; ++j) {
                            const int a = (WAVE + STR * j) / 3;
                            const float4 w = *(const float4 *)(wx + a * SW + 16 * pk + 4 * u);
                            nw[j][0] = w.x; nw[j][1] = w.y; nw[j][2] = w.z; nw[j][3] = w.w;
                        }
                    }
                };
                load(0);
                // FP64: no unrolling across groups (its accumulators and FP64
                // sums leave no room for a second group's operands)
#pragma unroll (PREC == ARGUS_FP32 ? 4 : 1)
                for (int u = 0; u < 4; ++u) {
                    const float ca[4] = {na.x, na.y, na.z, na.w};
                    const float cb[4] = {nb.x, nb.y, nb.z, nb.w};
                    const float cz[4] = {nz.x, nz.y, nz.z, nz.w};
                    T w[NTW][4];
                    if constexpr (PREC == ARGUS_FP32) {
#pragma unroll
                        for (int j = 0; j < NTW; ++j)
#pragma unroll
                            for (int e = 0; e < 4; ++e) w[j][e] = nw[j][e];
                    } else {
#pragma unroll
                        for (int j = 0; j < NTW; ++j) {
                            const int a = (WAVE + STR * j) / 3;
                            const double2 w0 = *(const double2 *)(wxd + a * SW + 16 * pk + 4 * u);
                            const double2 w1 = *(const double2 *)(wxd + a * SW + 16 * pk + 4 * u + 2);
                            w[j][0] = w0.x; w[j][1] = w0.y; w[j][2] = w1.x; w[j][3] = w1.y;
                        }
                    }
                    if (u + 1 < 4) load(u + 1);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const T c0 = (T)ca[e] + (T)g0 * (T)cz[e];
                        const T c1 = (T)cb[e] + (T)g1 * (T)cz[e];
#pragma unroll
                        for (int j = 0; j < NTW; ++j) {
                            const int bp = (WAVE + STR * j) % 3;
                            const T A = (bp == 2) ? c1 : c0;
                            const T B = w[j][e] * ((bp == 0) ? c0 : c1);
                            if constexpr (PREC == ARGUS_FP32)
                                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(A, B, acc[j], 0, 0, 0);
                            else
                                acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(A, B, acc[j], 0, 0, 0);
                        }
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < NTW; ++j) acc[j] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < SW / 32; ++s) {
                    const int p0 = 32 * s + 8 * pk;          // this lane's 8 pixels
                    float c0[8], c1[8];
                    bf16x8 h0, l0, h1, l1;
                    {
                        const float4 a0 = *(const float4 *)(cvec + col * CKM + p0);
                        const float4 a1 = *(const float4 *)(cvec + col * CKM + p0 + 4);
                        const float4 b0 = *(const float4 *)(cvec + (16 + col) * CKM + p0);
                        const float4 b1 = *(const float4 *)(cvec + (16 + col) * CKM + p0 + 4);
                        const float4 z0 = *(const float4 *)(cvec + p0);
                        const float4 z1 = *(const float4 *)(cvec + p0 + 4);
                        const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
                        const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
                        const float zv[8] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w};
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            c0[e] = av[e] + g0 * zv[e];
                            c1[e] = bv[e] + g1 * zv[e];
                            const __bf16 x0 = (__bf16)c0[e], x1 = (__bf16)c1[e];
                            h0[e] = x0;
                            l0[e] = (__bf16)(c0[e] - (float)x0);
                            h1[e] = x1;
                            l1[e] = (__bf16)(c1[e] - (float)x1);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < NTW; ++j) {
                        const int t = WAVE + STR * j;
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
    }

    __device__ void row_km(const float *cvec, const float *wx, const double *wxd,
                           const double *ypw, int lane, float g0, float g1) {
        Acc acc[NTW > 0 ? NTW : 1];
        row_km_acc(cvec, wx, wxd, lane, g0, g1, acc);
        flush(acc, ypw);
    }

    // Output element of register r in this lane: column lane % 16; row
    // 4 (lane / 16) + r for the FP32 and BF16 instructions, 4 r + lane / 16 for
    // v_mfma_f64_16x16x4f64.
    __device__ void store(double *part, int lane) {
        if constexpr (NTW > 0) {
            const int col = lane & 15, lg = lane >> 4;
#pragma unroll
            for (int j = 0; j < NTW; ++j) {
                const int t = WAVE + STR * j;
                const int a = t / 3, bp = t % 3;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (b <= 2 * D - a) {
                        double *g = part + (size_t)qidx(a, b, 2 * D) * 768 + bp * 256;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = (PREC == ARGUS_FP64) ? 4 * r + lg : 4 * lg + r;
                            g[row * 16 + col] = F[j][b][r];
                        }
                    }
                }
            }
        }
    }
};

// Wave-uniform loads of the filter tables go through the scalar cache.
typedef const __attribute__((address_space(4))) float *cfloat_p;
__device__ __forceinline__ float uload(const float *p) { return *(cfloat_p)p; }

// LDS carve-up of the accumulation kernel (4-byte words).
template <int D, int HH>
struct FitLds {
    static constexpr int K = 2 * HH + 1;
    static constexpr int IN = SW + 2 * HH;               // input row length
    static constexpr int INP = (IN + 3) & ~3;
    float *rowbuf, *inrow, *cvec, *wx, *wsx;
    double *wxd, *wsxd;
    uint8_t *minrow;
    __host__ __device__ static size_t bytes(int nplanes) {
        using S = FitShape<D>;
        size_t w = (size_t)nplanes * K * SW + 2 * INP + SW * CST + (S::NA + S::NRA) * SW;
        size_t b = w * 4 + (size_t)(S::NA + S::NRA) * SW * 8 + 2 * INP + 16;
        size_t rhs = (size_t)8 * S::NR * 32 * 8 + 256;    // end-of-kernel reuse of rowbuf
        return (b > rhs ? b : rhs) + 64;
    }
    __device__ FitLds(float *lds, int nplanes) {
        using S = FitShape<D>;
        rowbuf = lds;                                   // [NPL][K][SW]: thread-private columns
        inrow = rowbuf + (size_t)nplanes * K * SW;      // [2][INP] double-buffered input row
        cvec = inrow + 2 * INP;                         // [SW][CST] raw basis convolutions
        wx = cvec + SW * CST;                           // [NA][SW]  w xt^a
        wsx = wx + S::NA * SW;                          // [NRA][SW] w S xt^a
        // wsx ends on a 16-byte boundary (INP, SW multiples of 4); no integer
        // round trip, which would make the LDS pointers generic
        wxd = (double *)(wsx + S::NRA * SW);            // [NA][SW]
        wsxd = wxd + S::NA * SW;                        // [NRA][SW] w S xt^a (FP64 path)
        minrow = (uint8_t *)(wsxd + S::NRA * SW);       // [2][INP] ref mask != 0
    }
};

// One workgroup: a 64-column strip of a region, rows [ry0, ry1).  Wave w owns
// the row-filter planes w, w+4, w+8, w+12 at column x = lane (its slice of the
// circular row buffer is private, so the row and column passes need no
// barrier between them); wave 0 also owns the fit-set weights.  Per input row:
// write the prefetched row to LDS, prefetch the next one, barrier, row filters,
// column filters + weights, barrier, MFMA moments and rhs of the output row.
template <int D, int HH, int WAVE, int PREC>
__device__ void fit_wave(const FitArgs &a, float *lds, int sx_begin, int sx_end, int ry0,
                         int ry1, bool active, double *part) {
    using S = FitShape<D>;
    using L = FitLds<D, HH>;
    constexpr int K = L::K;
    const int tid = threadIdx.x, lane = tid & 63;
    const int NPL = a.nplanes;
    L l(lds, NPL);
    double *rhsbuf = (double *)lds;

    WaveGram<D, WAVE, PREC> gram;
    gram.zero();
    double RF[S::NR];
#pragma unroll
    for (int i = 0; i < S::NR; ++i) RF[i] = 0.0;
    int count = 0;

    // this wave's planes (wave-uniform)
    int k0[4], nk[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int p = a.plist[WAVE][j];
        k0[j] = 0;
        nk[j] = 0;
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
    const float g0 = (lane & 15) < a.nb ? a.tab->gam[lane & 15] : 0.f;
    const float g1 = 16 + (lane & 15) < a.nb ? a.tab->gam[16 + (lane & 15)] : 0.f;
    const float gk = (lane & 31) < a.nb ? a.tab->gam[lane & 31] : 0.f;  // rhs fix-up
    // strips of SW columns over [sx_begin, sx_end); the sums run across strips
    const int nstrips = active ? (sx_end - sx_begin + SW - 1) / SW : 1;
    for (int strip = 0; strip < nstrips; ++strip) {
    const int sx0 = sx_begin + strip * SW, sx1 = min(sx0 + SW, sx_end);
    const double xtd = (double)(sx0 + lane) * a.sx - (a.sx != 0.0 ? 1.0 : 0.0);
    const float xt = (float)xtd;

    const int64_t P = a.pitch;
    // prefetch registers: input row element (threads < IN) and the weight inputs
    float pr = 0.f;
    uint8_t pm = 0;
    float p_s = 0.f, p_sv = 0.f, p_rv = 0.f;
    uint8_t p_sm = 1;
    // the prefetches only load (from clamped addresses); the selects happen
    // where the values are used, so the loads stay in flight for a row
    bool pin = false, pok = false;
    const int Xin = sx0 - HH + tid;
    const bool in_x = tid < L::IN && Xin >= 0 && Xin < a.W;
    const int Xc = in_x ? Xin : (Xin < 0 ? 0 : a.W - 1);
    auto fetch_in = [&](int yy) {
        if (tid < L::IN) {
            // (global loads: the batch builds these arguments from a frame
            // table, where the compiler cannot see the address space)
            pr = gld(a.ref + (int64_t)yy * P + Xc);
            pm = gld(a.rmask + (int64_t)yy * P + Xc);
            pin = in_x;
        }
    };
    const bool lane_ok = sx0 + lane < sx1;
    const int64_t xw = lane_ok ? sx0 + lane : sx0;
    auto fetch_w = [&](int y) {
        if (WAVE == 0) {
            pok = lane_ok && y >= ry0 && y < ry1;
            const int yc = y < ry1 ? y : ry1 - 1;
            const int64_t o = (int64_t)yc * P + xw;
            p_s = gld(a.sci + o);
            p_sv = gld(a.svar + o);
            p_rv = gld(a.rvar + o);
            p_sm = gld(a.smask + o);
        }
    };
    uint32_t hist = 0;                     // bit j: input row yy-j has a flagged pixel in reach
    const int yend = active ? ry1 + HH : ry0 - HH;
    if (active) {
        fetch_in(ry0 - HH);
        fetch_w(ry0);
    }
    for (int yy = ry0 - HH; yy < yend; ++yy) {
        const int buf = yy & 1;
        if (tid < L::IN) {
            l.inrow[buf * L::INP + tid] = pin ? pr : 0.f;
            l.minrow[buf * L::INP + tid] = (pin && pm != 0) ? 1 : 0;
        }
        const float w_s = p_s, w_sv = p_sv, w_rv = p_rv;
        const uint8_t w_sm = pok ? p_sm : 1;
        if (yy + 1 < yend) fetch_in(yy + 1);
        const bool outrow = yy >= ry0 + HH;
        if (outrow) fetch_w(yy + 1 - HH);
        __syncthreads();
        // row filters of my planes at x = lane
        const int slot = yy % K;
        {
            float win[K];
            const float *ir = l.inrow + buf * L::INP + lane;
#pragma unroll
            for (int uu = 0; uu < K; ++uu) win[uu] = ir[2 * HH - uu];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int p = a.plist[WAVE][j];
                if (p >= 0) {
                    const float *f = &a.tab->rowf[p][0];
                    float acc = 0.f;
#pragma unroll
                    for (int uu = 0; uu < K; ++uu) acc += uload(f + uu) * win[uu];
                    l.rowbuf[((size_t)p * K + slot) * SW + lane] = acc;
                }
            }
            if (WAVE == 0) {
                const uint8_t *mr = l.minrow + buf * L::INP + lane;
                uint8_t m = 0;
#pragma unroll
                for (int uu = 0; uu < K; ++uu) m |= mr[uu];
                hist = (hist << 1) | (m ? 1u : 0u);
            }
        }
        if (outrow) {
            const int y = yy - HH;
            // column filters: rows y-h..y+h sit in slots (yy+1 .. yy+K) mod K
            int s0 = (yy + 1) % K;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int p = a.plist[WAVE][j];
                if (p >= 0) {
                    float t[K];
#pragma unroll
                    for (int jj = 0; jj < K; ++jj) {
                        int sl = s0 + jj;
                        sl -= sl >= K ? K : 0;
                        t[jj] = l.rowbuf[((size_t)p * K + sl) * SW + lane];
                    }
#pragma unroll
                    for (int q = 0; q < 7; ++q) {
                        if (q < nk[j]) {
                            const float *f = &a.tab->colf[k0[j] + q][0];
                            float acc = 0.f;
#pragma unroll
                            for (int jj = 0; jj < K; ++jj) acc += uload(f + 2 * HH - jj) * t[jj];
                            l.cvec[lane * CST + k0[j] + q] = acc;
                        }
                    }
                }
            }
            if (WAVE == 0) {
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
                    l.wx[e * SW + lane] = w * xp;
                    if (PREC == ARGUS_FP64) l.wxd[e * SW + lane] = (double)w * xpd;
                    if (e < S::NRA) l.wsx[e * SW + lane] = w * w_s * xp;
                    if (PREC == ARGUS_FP64 && e < S::NRA)
                        l.wsxd[e * SW + lane] = (double)w * (double)w_s * xpd;
                    xp *= xt;
                    xpd *= xtd;
                }
            }
        }
        __syncthreads();
        if (outrow) {
            const int y = yy - HH;
            double ypw[2 * D + 1];
            {
                double yt = (double)y * a.sy - (a.sy != 0.0 ? 1.0 : 0.0);
                double yp = 1.0;
#pragma unroll
                for (int b = 0; b <= 2 * D; ++b) { ypw[b] = yp; yp *= yt; }
            }
            gram.row(l.cvec, l.wx, l.wxd, ypw, lane, g0, g1);
            {
                const int k = lane & 31, half = lane >> 5;
                if constexpr (PREC == ARGUS_FP64) {
                    // right-hand side in FP64: products and the 8-pixel sums
                    double ra[S::NRA];
#pragma unroll
                    for (int e = 0; e < S::NRA; ++e) ra[e] = 0.0;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int px = WAVE * 16 + half * 8 + i;
                        const double c = (double)l.cvec[px * CST + k] +
                                         (double)gk * (double)l.cvec[px * CST];
#pragma unroll
                        for (int e = 0; e < S::NRA; ++e) ra[e] += l.wsxd[e * SW + px] * c;
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
                    for (int i = 0; i < 8; ++i) {
                        const int px = WAVE * 16 + half * 8 + i;
                        const float c = l.cvec[px * CST + k] + gk * l.cvec[px * CST];
#pragma unroll
                        for (int e = 0; e < S::NRA; ++e) ra[e] += l.wsx[e * SW + px] * c;
                    }
#pragma unroll
                    for (int e = 0; e < S::NRA; ++e)
#pragma unroll
                        for (int b = 0; b <= D; ++b)
                            if (e + b <= D) RF[qidx(e, b, D)] += ypw[b] * (double)ra[e];
                }
            }
        }
    }
    }
    __syncthreads();
    gram.store(part, lane);
    {
        const int k = lane & 31, half = lane >> 5;
#pragma unroll
        for (int i = 0; i < S::NR; ++i) rhsbuf[((WAVE * 2 + half) * S::NR + i) * 32 + k] = RF[i];
    }
    if (WAVE == 0) {
        double c = (double)count;
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
        if (lane == 0) part[(size_t)S::NQ * 768 + S::NR * 32] = c;
    }
    __syncthreads();
    for (int it = tid; it < S::NR * 32; it += NTHR) {
        double s = 0.0;
        for (int q = 0; q < 8; ++q) s += rhsbuf[q * S::NR * 32 + it];
        part[(size_t)S::NQ * 768 + it] = s;
    }
}

template <int D, int HH, int PREC>
__global__ __launch_bounds__(NTHR) void fit_accum_kernel(FitArgs a) {
    extern __shared__ float lds[];
    const int tid = threadIdx.x;
    // workgroup -> region, strip, row chunk
    const int s = blockIdx.x % a.spt, rx = blockIdx.x / a.spt;
    const int rc = blockIdx.y % a.rchunks, ry = blockIdx.y / a.rchunks;
    const int rx0 = (int)((int64_t)rx * a.W / a.RX), rx1 = (int)((int64_t)(rx + 1) * a.W / a.RX);
    const int ry0g = (int)((int64_t)ry * a.H / a.RY), ry1g = (int)((int64_t)(ry + 1) * a.H / a.RY);
    const int ix0 = max(rx0, HH), ix1 = min(rx1, a.W - HH);
    const int iy0 = max(ry0g, HH), iy1 = min(ry1g, a.H - HH);
    int sx0 = ix0 + s * SW, sx1 = min(sx0 + SW, ix1);
    int rows = max(iy1 - iy0, 0);
    int rh = (rows + a.rchunks - 1) / a.rchunks;
    int ry0 = iy0 + rc * rh, ry1 = min(ry0 + rh, iy1);
    const bool active = sx0 < sx1 && ry0 < ry1;    // otherwise the partial is all zeros
    const int pid = ((ry * a.RX + rx) * a.rchunks + rc) * a.spt + s;
    double *part = a.partials + (size_t)pid * a.stride;
    // constant tail of c: 1 at index nb (background), zeros after
    FitLds<D, HH> L(lds, a.nplanes);
    for (int i = tid; i < SW * CST; i += NTHR) {
        int k = i % CST;
        if (k >= a.nb) L.cvec[i] = (k == a.nb) ? 1.f : 0.f;
    }
    switch (tid >> 6) {
        case 0: fit_wave<D, HH, 0, PREC>(a, lds, sx0, sx1, ry0, ry1, active, part); break;
        case 1: fit_wave<D, HH, 1, PREC>(a, lds, sx0, sx1, ry0, ry1, active, part); break;
        case 2: fit_wave<D, HH, 2, PREC>(a, lds, sx0, sx1, ry0, ry1, active, part); break;
        default: fit_wave<D, HH, 3, PREC>(a, lds, sx0, sx1, ry0, ry1, active, part); break;
    }
}


// Launch fit_accum_kernel<D, h, PREC> with its dynamic LDS size.
template <int PREC>
int fit_accum_launch(argus_ctx *ctx, const FitArgs &fa, int D, dim3 grid) {
    hipError_t err = hipSuccess;
    bool ok = false;
#define ARGUS_FH(DD, HH)                                                                   \
    if (D == DD && fa.h == HH) {                                                           \
        size_t lds = FitLds<DD, HH>::bytes(fa.nplanes);                                    \
        err = hipFuncSetAttribute((const void *)fit_accum_kernel<DD, HH, PREC>,            \
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        if (err == hipSuccess)                                                             \
            hipLaunchKernelGGL((fit_accum_kernel<DD, HH, PREC>), grid, dim3(NTHR), lds,    \
                               ctx->stream, fa);                                           \
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

// One launcher per precision, each in its own translation unit.
int fit_accum_launch_fp32(argus_ctx *ctx, const argus_fit::FitArgs &fa, int D, dim3 grid);
int fit_accum_launch_fp64(argus_ctx *ctx, const argus_fit::FitArgs &fa, int D, dim3 grid);
int fit_accum_launch_bf16x3(argus_ctx *ctx, const argus_fit::FitArgs &fa, int D, dim3 grid);
