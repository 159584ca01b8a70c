// PSF-matched convolution of the reference, subtraction from the science
// frame, propagated variance and the fit-set chi^2.
//
// Per output pixel p the kernel is evaluated at p (K_p = sum_m P_m(p) K_m).
// Along a row yt is fixed, so with the stamps ordered (p,q) = (0,0),(0,1),
// (0,2),(1,0),(1,1),(2,0):  K_p = A0 + xt (A1 + xt A2), A0 = K0 + yt (K1 +
// yt K2), A1 = K3 + yt K4, A2 = K5.  A thread owns 8 consecutive pixels of a
// row: the A's of a tap are evaluated once for its row and shared by the 8
// pixels, the reference and variance windows of a kernel row sit in
// registers, and each tap costs 5 VALU ops per pixel (2 for a constant
// kernel).  Workgroups are 128x16 output pixels with an h-pixel halo in LDS.
#include <mutex>

#include "internal.h"

// Block partials of argus_subtract_noalloc: a fixed device array, so that
// entry point allocates nothing.  Host code never passes the name itself to a
// kernel (it stands for a host-side shadow); it passes the device address
// fetched once per device by subtract_scratch_init.
static __device__ __align__(256) double scratch[(size_t)ARGUS_NOALLOC_MAX_BLOCKS * 4];

namespace {

constexpr int BW = 128, BH = 16, PXT = 8, NTHR = 256;

struct SubArgs {
    const float *stamps, *bg;
    const float *ref, *rvar, *sci, *svar;
    const uint8_t *rmask, *smask;
    float *diff, *dvar;
    uint8_t *dmask;
    double *partials;          // [n_blocks][4]: chi^2, count, sum w D, sum w
    int64_t pitch;
    int W, H, D, Dbg;
    int RX, RY, bpx, bpy;      // regions and blocks per region
    double sx, sy;
    int vec;
    int write;                 // 0: only the sums (diff, dvar, dmask are null)
};

template <int HH>
struct SubLds {
    static constexpr int K = 2 * HH + 1;
    static constexpr int TH = BH + 2 * HH;
    static constexpr int TWr = BW + 2 * HH;
    static constexpr int TW = (TWr + 3) & ~3;          // float row stride, 16-byte aligned
    static constexpr int MW = (TWr + 15) & ~15;         // mask row stride
};

template <int D, int HH>
__global__ __launch_bounds__(NTHR) void subtract_kernel(SubArgs a) {
    using L = SubLds<HH>;
    constexpr int K = L::K, TH = L::TH, TW = L::TW, MW = L::MW, NP = (D + 1) * (D + 2) / 2;
    constexpr int NS = (D == 0) ? 2 : NP;               // constant kernel also keeps K^2
    constexpr int NSP = NS <= 4 ? 4 : 8;                // per-tap values, padded to 16-byte reads
    extern __shared__ float lds[];
    float *Rt = lds;                                    // [TH][TW]
    float *Vt = Rt + TH * TW;                           // [TH][TW]
    float *St = Vt + TH * TW;                           // [K*K][NSP] stamp values per tap
    uint8_t *Mt = (uint8_t *)(St + NSP * K * K);        // [TH][MW] ref mask != 0
    uint8_t *Mr = Mt + TH * MW;                         // [TH][BW] row-OR over 2h+1
    __shared__ double red[4][NTHR / 64];

    const int tid = threadIdx.x;
    const int bid = blockIdx.x;
    const int bx = bid % a.bpx;
    const int by = (bid / a.bpx) % a.bpy;
    const int reg = bid / (a.bpx * a.bpy);
    const int rx = reg % a.RX, ry = reg / a.RX;
    const int rx0 = (int)((int64_t)rx * a.W / a.RX), rx1 = (int)((int64_t)(rx + 1) * a.W / a.RX);
    const int ry0 = (int)((int64_t)ry * a.H / a.RY), ry1 = (int)((int64_t)(ry + 1) * a.H / a.RY);
    const int bx0 = rx0 + bx * BW, by0 = ry0 + by * BH;
    const int bx1 = min(bx0 + BW, rx1), by1 = min(by0 + BH, ry1);
    const int64_t P = a.pitch;

    double c2 = 0.0, cnt = 0.0, swd = 0.0, sw = 0.0;
    if (bx0 < bx1 && by0 < by1) {
        // halo tiles of the reference, its variance and mask: every load of a
        // thread is issued before any is used (clamped addresses, the
        // out-of-frame zeros applied at the store), so they are all in flight
        // together instead of one latency per element
        {
            constexpr int NH = (TH * L::TWr + NTHR - 1) / NTHR, NB8 = 8;
            for (int j0 = 0; j0 < NH; j0 += NB8) {       // 8 elements in flight per batch
                float hr[NB8], hv[NB8];
                uint8_t hm[NB8];
#pragma unroll
                for (int j = 0; j < NB8; ++j) {
                    const int i = tid + (j0 + j) * NTHR;
                    const int ii = i < TH * L::TWr ? i : 0;
                    const int cy = ii / L::TWr, cx = ii % L::TWr;
                    int X = bx0 - HH + cx, Y = by0 - HH + cy;
                    X = X < 0 ? 0 : (X >= a.W ? a.W - 1 : X);
                    Y = Y < 0 ? 0 : (Y >= a.H ? a.H - 1 : Y);
                    const int64_t o = (int64_t)Y * P + X;
                    hr[j] = a.ref[o];
                    hv[j] = a.rvar[o];
                    hm[j] = a.rmask[o];
                }
#pragma unroll
                for (int j = 0; j < NB8; ++j) {
                    const int i = tid + (j0 + j) * NTHR;
                    if (i < TH * L::TWr) {
                        const int cy = i / L::TWr, cx = i % L::TWr;
                        const int X = bx0 - HH + cx, Y = by0 - HH + cy;
                        const bool in = X >= 0 && X < a.W && Y >= 0 && Y < a.H;
                        Rt[cy * TW + cx] = in ? hr[j] : 0.f;
                        Vt[cy * TW + cx] = in ? hv[j] : 0.f;
                        Mt[cy * MW + cx] = (in && hm[j] != 0) ? 1 : 0;
                    }
                }
            }
        }
        const float *src = a.stamps + (size_t)reg * NP * K * K;
        {
            constexpr int NS_ = (NP * K * K + NTHR - 1) / NTHR;
            float sv_[NS_];
#pragma unroll
            for (int j = 0; j < NS_; ++j) {
                const int i = tid + j * NTHR;
                sv_[j] = src[i < NP * K * K ? i : 0];
            }
#pragma unroll
            for (int j = 0; j < NS_; ++j) {
                const int i = tid + j * NTHR;
                if (i < NP * K * K) {
                    const int t = i % (K * K), m = i / (K * K);
                    St[t * NSP + m] = sv_[j];
                    if (D == 0) St[t * NSP + 1] = sv_[j] * sv_[j];
                }
            }
        }
        __syncthreads();
        for (int i = tid; i < TH * (BW / PXT); i += NTHR) {
            int cy = i / (BW / PXT), lx0 = (i % (BW / PXT)) * PXT;
            uint8_t w[PXT + 2 * HH];
#pragma unroll
            for (int j = 0; j < PXT + 2 * HH; ++j) w[j] = Mt[cy * MW + lx0 + j];
#pragma unroll
            for (int px = 0; px < PXT; ++px) {
                uint8_t m = 0;
#pragma unroll
                for (int uu = 0; uu < K; ++uu) m |= w[px + uu];
                Mr[cy * BW + lx0 + px] = m;
            }
        }
        __syncthreads();

        const int ly = tid / (BW / PXT), lx0 = (tid % (BW / PXT)) * PXT;
        const int Y = by0 + ly;
        float xt[PXT];
#pragma unroll
        for (int i = 0; i < PXT; ++i)
            xt[i] = (float)((double)(bx0 + lx0 + i) * a.sx - (a.sx != 0.0 ? 1.0 : 0.0));
        const double ytd = (double)Y * a.sy - (a.sy != 0.0 ? 1.0 : 0.0);
        const float yt = (float)ytd;
        float m[PXT], v[PXT];
#pragma unroll
        for (int i = 0; i < PXT; ++i) { m[i] = 0.f; v[i] = 0.f; }
        if (Y < by1) {
            for (int vv = 0; vv < K; ++vv) {
                // the windows of this kernel row as 16-byte reads (rows are
                // 16-byte aligned; the last read may pass the window by two
                // floats, inside the row)
                constexpr int NW4 = (PXT + 2 * HH + 3) / 4;
                const float4 *rr = (const float4 *)(Rt + (ly + 2 * HH - vv) * TW + lx0);
                const float4 *qq = (const float4 *)(Vt + (ly + 2 * HH - vv) * TW + lx0);
                float r[4 * NW4], q[4 * NW4];
#pragma unroll
                for (int j = 0; j < NW4; ++j) {
                    const float4 a4 = rr[j], b4 = qq[j];
                    r[4 * j] = a4.x; r[4 * j + 1] = a4.y; r[4 * j + 2] = a4.z; r[4 * j + 3] = a4.w;
                    q[4 * j] = b4.x; q[4 * j + 1] = b4.y; q[4 * j + 2] = b4.z; q[4 * j + 3] = b4.w;
                }
#pragma unroll
                for (int uu = 0; uu < K; ++uu) {
                    // this tap's stamp values, one or two 16-byte reads
                    float st[NSP];
                    {
                        const float4 *sp = (const float4 *)(St + (vv * K + uu) * NSP);
#pragma unroll
                        for (int e = 0; e < NSP / 4; ++e) {
                            const float4 v4 = sp[e];
                            st[4 * e] = v4.x; st[4 * e + 1] = v4.y; st[4 * e + 2] = v4.z; st[4 * e + 3] = v4.w;
                        }
                    }
                    if constexpr (D == 0) {
                        const float k = st[0], k2 = st[1];
#pragma unroll
                        for (int i = 0; i < PXT; ++i) {
                            m[i] += k * r[i + 2 * HH - uu];
                            v[i] += k2 * q[i + 2 * HH - uu];
                        }
                    } else if constexpr (D == 1) {
                        const float A0 = st[0] + yt * st[1];
                        const float A1 = st[2];
#pragma unroll
                        for (int i = 0; i < PXT; ++i) {
                            const float k = A0 + xt[i] * A1;
                            m[i] += k * r[i + 2 * HH - uu];
                            v[i] += (k * k) * q[i + 2 * HH - uu];
                        }
                    } else {
                        const float A0 = st[0] + yt * (st[1] + yt * st[2]);
                        const float A1 = st[3] + yt * st[4];
                        const float A2 = st[5];
#pragma unroll
                        for (int i = 0; i < PXT; ++i) {
                            const float k = A0 + xt[i] * (A1 + xt[i] * A2);
                            m[i] += k * r[i + 2 * HH - uu];
                            v[i] += (k * k) * q[i + 2 * HH - uu];
                        }
                    }
                }
            }
            // footprint flags from the row-ORed mask
            uint8_t foot[PXT];
#pragma unroll
            for (int i = 0; i < PXT; ++i) foot[i] = 0;
            for (int vv = 0; vv < K; ++vv) {
#pragma unroll
                for (int i = 0; i < PXT; ++i) foot[i] |= Mr[(ly + vv) * BW + lx0 + i];
            }
            // background polynomial of this pixel's solve, folded along the row
            // (yt fixed) into x-coefficients: bg = sum_p cx[p] xt^p with
            // cx[p] = sum_q bg_pq yt^q (monomials p outer, q inner)
            const float *bgp = a.bg + (size_t)reg * ((a.Dbg + 1) * (a.Dbg + 2) / 2);
            double cx[ARGUS_MAX_D + 1];
            {
                int mi = 0;
#pragma unroll
                for (int pp = 0; pp <= ARGUS_MAX_D; ++pp) {
                    double c = 0.0, yq = 1.0;
                    for (int qq = 0; pp <= a.Dbg && qq <= a.Dbg - pp; ++qq, ++mi) {
                        c += (double)bgp[mi] * yq;
                        yq *= ytd;
                    }
                    cx[pp] = c;
                }
            }
            float outd[PXT], outv[PXT];
            uint8_t outm[PXT];
            const int64_t orow = (int64_t)Y * P;
#pragma unroll
            for (int i = 0; i < PXT; ++i) {
                const int X = bx0 + lx0 + i;
                outd[i] = 0.f; outv[i] = 0.f; outm[i] = 0;
                if (X < bx1) {
                    const int64_t o = orow + X;
                    const bool edge = X < HH || X > a.W - 1 - HH || Y < HH || Y > a.H - 1 - HH;
                    uint8_t dm = a.smask[o] | (edge ? ARGUS_EDGE : 0u) |
                                 ((!edge && foot[i]) ? ARGUS_FOOT : 0u);
                    outm[i] = dm;
                    if (dm == 0) {
                        const double xd = (double)X * a.sx - (a.sx != 0.0 ? 1.0 : 0.0);
                        double bgv = cx[ARGUS_MAX_D];
#pragma unroll
                        for (int pp = ARGUS_MAX_D - 1; pp >= 0; --pp) bgv = bgv * xd + cx[pp];
                        const float s = a.sci[o], sv = a.svar[o];
                        const float dval = s - (float)((double)m[i] + bgv);
                        outd[i] = dval;
                        outv[i] = sv + v[i];
                        const float tot = sv + a.rvar[o];
                        if (tot > 0.f) {
                            const double w = 1.0 / (double)tot, wd = w * (double)dval;
                            c2 += wd * (double)dval;
                            cnt += 1.0;
                            swd += wd;
                            sw += w;
                        }
                    }
                }
            }
            const int X0 = bx0 + lx0;
            const int64_t o0 = orow + X0;
            if (!a.write) {
                // chi^2 pass of the fit: no images written
            } else if (a.vec && (X0 & 7) == 0 && X0 + PXT <= bx1) {
                *(float4 *)(a.diff + o0) = make_float4(outd[0], outd[1], outd[2], outd[3]);
                *(float4 *)(a.diff + o0 + 4) = make_float4(outd[4], outd[5], outd[6], outd[7]);
                *(float4 *)(a.dvar + o0) = make_float4(outv[0], outv[1], outv[2], outv[3]);
                *(float4 *)(a.dvar + o0 + 4) = make_float4(outv[4], outv[5], outv[6], outv[7]);
                uint2 mo;
                mo.x = outm[0] | (outm[1] << 8) | (outm[2] << 16) | ((uint32_t)outm[3] << 24);
                mo.y = outm[4] | (outm[5] << 8) | (outm[6] << 16) | ((uint32_t)outm[7] << 24);
                *(uint2 *)(a.dmask + o0) = mo;
            } else {
#pragma unroll
                for (int i = 0; i < PXT; ++i) {
                    if (X0 + i < bx1) {
                        a.diff[o0 + i] = outd[i];
                        a.dvar[o0 + i] = outv[i];
                        a.dmask[o0 + i] = outm[i];
                    }
                }
            }
        }
    }
    // fixed-order block reduction of chi^2, the fit-set count, sum w D, sum w
    for (int off = 32; off > 0; off >>= 1) {
        c2 += __shfl_xor(c2, off);
        cnt += __shfl_xor(cnt, off);
        swd += __shfl_xor(swd, off);
        sw += __shfl_xor(sw, off);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = c2; red[1][tid >> 6] = cnt; red[2][tid >> 6] = swd; red[3][tid >> 6] = sw;
    }
    __syncthreads();
    if (tid < 4) {
        double sc = 0.0;
        for (int i = 0; i < NTHR / 64; ++i) sc += red[tid][i];
        a.partials[4 * (size_t)bid + tid] = sc;
    }
}

// One workgroup (256 threads) per solve: fixed-order sum of its blocks' partials.
__global__ void chi2_reduce_kernel(const double *part, int per_solve, double *chi2, int64_t *n,
                                   double *sum_wd, double *sum_w) {
    __shared__ double rs[4][4];
    const int s = blockIdx.x, tid = threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = tid; j < per_solve; j += blockDim.x) {
        const double *q = part + 4 * ((size_t)s * per_solve + j);
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] += q[c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off);
    if ((tid & 63) == 0)
#pragma unroll
        for (int c = 0; c < 4; ++c) rs[c][tid >> 6] = v[c];
    __syncthreads();
    if (tid == 0) {
        double t[4];
        for (int c = 0; c < 4; ++c) {
            t[c] = 0.0;
            for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t[c] += rs[c][i];
        }
        if (chi2) chi2[s] = t[0];
        if (n) n[s] = (int64_t)t[1];
        if (sum_wd) sum_wd[s] = t[2];
        if (sum_w) sum_w[s] = t[3];
    }
}

template <int D, int HH>
int sub_launch(argus_ctx *ctx, SubArgs &a, int n_blocks) {
    using L = SubLds<HH>;
    constexpr int NP = (D + 1) * (D + 2) / 2;
    constexpr int NS = (D == 0) ? 2 : NP;
    constexpr int NSP = NS <= 4 ? 4 : 8;
    size_t lds = (size_t)2 * L::TH * L::TW * 4 + (size_t)NSP * L::K * L::K * 4 +
                 (size_t)L::TH * L::MW + (size_t)L::TH * BW;
    ARGUS_HIP_CHECK(ctx, hipFuncSetAttribute((const void *)subtract_kernel<D, HH>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((subtract_kernel<D, HH>), dim3(n_blocks), dim3(NTHR), lds, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

template <int D>
int sub_dispatch_h(argus_ctx *ctx, SubArgs &a, int h, int n_blocks) {
    switch (h) {
#define ARGUS_SH(HH) case HH: return sub_launch<D, HH>(ctx, a, n_blocks);
        ARGUS_SH(1) ARGUS_SH(2) ARGUS_SH(3) ARGUS_SH(4) ARGUS_SH(5) ARGUS_SH(6) ARGUS_SH(7)
        ARGUS_SH(8) ARGUS_SH(9) ARGUS_SH(10) ARGUS_SH(11) ARGUS_SH(12) ARGUS_SH(13)
        ARGUS_SH(14) ARGUS_SH(15)
#undef ARGUS_SH
        default: return argus_fail(ctx, ARGUS_ESHAPE, "half width %d unsupported", h);
    }
}

inline bool aligned(const void *p, size_t al) { return ((uintptr_t)p % al) == 0; }

}  // namespace

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[ARGUS_MAX_DEVICES] = {};
}  // namespace

int subtract_scratch_init(argus_ctx *ctx) {
    if (ctx->device < 0 || ctx->device >= ARGUS_MAX_DEVICES)
        return argus_fail(ctx, ARGUS_EINVAL, "device %d beyond the scratch table", ctx->device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[ctx->device]) return ARGUS_OK;
    // the caller made ctx->device current; each device has its own copy
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return argus_fail(ctx, ARGUS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[ctx->device] = (double *)p;
    return ARGUS_OK;
}

int launch_subtract(argus_ctx *ctx, argus_dims d, const argus_kernel_spec *spec,
                    const float *stamps, const float *bg, const float *ref,
                    const float *ref_var, const uint8_t *ref_mask, const float *sci,
                    const float *sci_var, const uint8_t *sci_mask, float *diff, float *diff_var,
                    uint8_t *diff_mask, double *chi2, int64_t *n_chi2, double *sum_wd,
                    double *sum_w, bool noalloc) {
    SubArgs a;
    a.stamps = stamps; a.bg = bg; a.ref = ref; a.rvar = ref_var; a.sci = sci; a.svar = sci_var;
    a.rmask = ref_mask; a.smask = sci_mask; a.diff = diff; a.dvar = diff_var; a.dmask = diff_mask;
    a.pitch = d.pitch; a.W = d.width; a.H = d.height;
    a.D = spec->spatial_degree; a.Dbg = spec->bg_degree;
    const bool global = spec->mode == ARGUS_FIT_GLOBAL;
    a.RX = global ? 1 : spec->tiles_x;
    a.RY = global ? 1 : spec->tiles_y;
    a.bpx = ((d.width + a.RX - 1) / a.RX + BW - 1) / BW;
    a.bpy = ((d.height + a.RY - 1) / a.RY + BH - 1) / BH;
    a.sx = d.width > 1 ? 2.0 / (d.width - 1) : 0.0;
    a.sy = d.height > 1 ? 2.0 / (d.height - 1) : 0.0;
    a.vec = (d.pitch % 8 == 0) && aligned(diff, 32) && aligned(diff_var, 32) && aligned(diff_mask, 8);
    a.write = diff != nullptr;
    const int n_solves = a.RX * a.RY;
    const int per_solve = a.bpx * a.bpy;
    const int n_blocks = n_solves * per_solve;
    int rc;
    if (noalloc) {
        if (n_blocks > ARGUS_NOALLOC_MAX_BLOCKS)
            return argus_fail(ctx, ARGUS_ESHAPE,
                              "argus_subtract_noalloc: %d blocks of 128x16 pixels exceed the "
                              "scratch maximum of %d", n_blocks, ARGUS_NOALLOC_MAX_BLOCKS);
        double *p = (ctx->device >= 0 && ctx->device < ARGUS_MAX_DEVICES)
                        ? g_scratch_ptr[ctx->device] : nullptr;
        if (!p) return argus_fail(ctx, ARGUS_EHIP, "scratch address not initialised");
        a.partials = p;
    } else {
        if ((rc = argus_ws_reserve(ctx, (size_t)n_blocks * 4 * sizeof(double) + 256))) return rc;
        a.partials = (double *)ctx->ws;
    }
    if (!noalloc) argus_time_begin(ctx);
    switch (a.D) {
        case 0: rc = sub_dispatch_h<0>(ctx, a, spec->half_width, n_blocks); break;
        case 1: rc = sub_dispatch_h<1>(ctx, a, spec->half_width, n_blocks); break;
        default: rc = sub_dispatch_h<2>(ctx, a, spec->half_width, n_blocks); break;
    }
    if (rc) return rc;
    if (!noalloc) argus_time_end(ctx, "subtract");
    if (chi2 || n_chi2 || sum_wd || sum_w) {
        hipLaunchKernelGGL(chi2_reduce_kernel, dim3(n_solves), dim3(256), 0, ctx->stream,
                           (const double *)a.partials, per_solve, chi2, n_chi2, sum_wd, sum_w);
        ARGUS_HIP_CHECK(ctx, hipGetLastError());
    }
    return ARGUS_OK;
}
