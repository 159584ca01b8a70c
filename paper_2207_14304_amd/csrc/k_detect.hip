// Detection on the difference image: noise-normalised map, threshold,
// raster-ordered local maxima, stable compaction, PSF-weighted fluxes.
//
// detect_map: one workgroup per 256 x 16 tile.  It forms the SNR of its rows
//   and one halo row/column on each side in LDS (4-pixel vector loads), writes
//   snr and det_mask (4-pixel vector stores) and counts the candidates of
//   each 256-pixel row segment.
// scan_tiles: exclusive scan of the segment counts within 1024-count tiles,
//   and each tile's total.
// detect_emit: a wave takes 64 segments (one scan tile's), adds the totals of
//   the tiles before theirs, and for each segment with candidates writes them
//   in raster order at their offsets and measures the PSF flux in FP64; the
//   first wave writes the candidate count.
//
// Source mode (argus_detect_sources): the same kernels on a calibrated frame,
// with D = cal - background evaluated from the filtered cell grid per pixel,
// V the calibration's variance and its mask; sources also get the centroid
// of max(D, 0) over the unmasked in-image 3 x 3 neighbourhood.
#include <algorithm>

#include "internal.h"
#include "background.h"

namespace {

constexpr int SEG = 256, ROWS = 16, NTHR = 256;   // a wave covers a 256-pixel row, 4 px a lane
constexpr int LW = SEG + 8;                        // LDS row: [3] = x0-1, [4..259], [260] = x0+256
constexpr int STILE = 1024;                        // counts per scan tile
static_assert(STILE % 64 == 0, "a wave's 64 segments lie in one scan tile");

struct DetArgs {
    const float *diff, *dvar;
    const uint8_t *dmask;
    float *snr;
    uint8_t *det;
    int32_t *counts;           // [nseg]   candidates per row segment
    int32_t *local;            // [nseg]   offset within its scan tile
    int32_t *tile_sum;         // [ntile]
    const float *psf;
    argus_candidate *cands;
    argus_source *srcs;
    int32_t *n_cands;
    BgGrid bg;                 // source mode: D = diff - bg(x, y)
    int64_t pitch;
    int W, H, nsx, nseg, ntile, r, cap;
    int vec;                   // 16-byte aligned planes, pitch % 4 == 0
    float thr;
};

// SNR of one pixel: D / sqrt(V) where the pixel is unmasked and V > 0, else 0;
// off-image pixels are -inf for the neighbour comparisons.
template <bool SRC>
__device__ __forceinline__ float d_at(const DetArgs &a, int64_t o, int x, int y) {
    if constexpr (SRC) return a.diff[o] - bg_at(a.bg, x, y);
    return a.diff[o];
}

template <bool SRC>
__device__ __forceinline__ float snr_at(const DetArgs &a, int x, int y) {
    if (x < 0 || x >= a.W || y < 0 || y >= a.H) return -__builtin_inff();
    int64_t o = (int64_t)y * a.pitch + x;
    float V = a.dvar[o];
    if (a.dmask[o] != 0 || !(V > 0.f)) return 0.f;
    return d_at<SRC>(a, o, x, y) * __builtin_amdgcn_rsqf(V);
}

__device__ __forceinline__ float snr_of(float D, float V, uint32_t m) {
    return (m != 0 || !(V > 0.f)) ? 0.f : D * __builtin_amdgcn_rsqf(V);
}

template <bool SRC>
__global__ __launch_bounds__(NTHR) void detect_map_kernel(DetArgs a) {
    __shared__ __align__(16) float s[ROWS + 2][LW];
    // tiles in raster order, each XCD a contiguous band of them (the halo rows
    // a tile shares with the tiles above and below stay in one L2)
    const int lb = argus_xcd_block((int)blockIdx.x, (int)gridDim.x);
    const int sx = lb % a.nsx, y0 = (lb / a.nsx) * ROWS, tid = threadIdx.x;
    const int x0 = sx * SEG;
    const int64_t P = a.pitch;
    // SNR of rows y0-1 .. y0+ROWS, 4-pixel chunks.  Vector path: all loads of
    // a thread are issued (from clamped rows) before any is used.
    constexpr int NCH = (ROWS + 2) * (SEG / 4), NIT = (NCH + NTHR - 1) / NTHR;
    if (a.vec && x0 + SEG <= a.W) {
        float4 Dv[NIT], Vv[NIT];
        uint32_t Mv[NIT];
#pragma unroll
        for (int j = 0; j < NIT; ++j) {
            const int i = tid + j * NTHR, ii = i < NCH ? i : 0;
            const int row = ii / (SEG / 4), ch = ii % (SEG / 4);
            int y = y0 - 1 + row;
            y = y < 0 ? 0 : (y >= a.H ? a.H - 1 : y);
            const int64_t o = (int64_t)y * P + x0 + 4 * ch;
            Dv[j] = *(const float4 *)(a.diff + o);
            Vv[j] = *(const float4 *)(a.dvar + o);
            Mv[j] = *(const uint32_t *)(a.dmask + o);
        }
#pragma unroll
        for (int j = 0; j < NIT; ++j) {
            const int i = tid + j * NTHR;
            if (i < NCH) {
                const int row = i / (SEG / 4), ch = i % (SEG / 4);
                const int y = y0 - 1 + row;
                float4 v;
                if (y < 0 || y >= a.H) {
                    v = make_float4(-__builtin_inff(), -__builtin_inff(), -__builtin_inff(),
                                    -__builtin_inff());
                } else {
                    float4 D = Dv[j];
                    const float4 V = Vv[j];
                    const uint32_t m = Mv[j];
                    if constexpr (SRC) {
                        const int x = x0 + 4 * ch;
                        D.x -= bg_at(a.bg, x, y);
                        D.y -= bg_at(a.bg, x + 1, y);
                        D.z -= bg_at(a.bg, x + 2, y);
                        D.w -= bg_at(a.bg, x + 3, y);
                    }
                    v = make_float4(snr_of(D.x, V.x, m & 0xffu),
                                    snr_of(D.y, V.y, (m >> 8) & 0xffu),
                                    snr_of(D.z, V.z, (m >> 16) & 0xffu),
                                    snr_of(D.w, V.w, m >> 24));
                }
                *(float4 *)&s[row][4 + 4 * ch] = v;
            }
        }
    } else {
        for (int i = tid; i < NCH; i += NTHR) {
            const int row = i / (SEG / 4), ch = i % (SEG / 4);
            const int y = y0 - 1 + row, x = x0 + 4 * ch;
            const float4 v = make_float4(snr_at<SRC>(a, x, y), snr_at<SRC>(a, x + 1, y),
                                         snr_at<SRC>(a, x + 2, y), snr_at<SRC>(a, x + 3, y));
            *(float4 *)&s[row][4 + 4 * ch] = v;
        }
    }
    if (tid < 2 * (ROWS + 2)) {
        const int row = tid >> 1, side = tid & 1;
        s[row][side ? 4 + SEG : 3] = snr_at<SRC>(a, side ? x0 + SEG : x0 - 1, y0 - 1 + row);
    }
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6;
    const int x = x0 + 4 * lane;
    for (int k = 0; k < ROWS / 4; ++k) {
        const int rr = w + 4 * k, y = y0 + rr;
        if (y >= a.H) break;                       // uniform across the wave
        // a lane's 4 pixels as one 16-byte read (consecutive lanes, no bank
        // conflicts), the neighbours from the adjacent lanes, the strip's two
        // edge values by broadcast reads
        auto row6 = [&](int r, float (&v)[6]) {
            const float4 c4 = *(const float4 *)&s[r][4 + 4 * lane];
            const float le = s[r][3], re = s[r][4 + SEG];
            const float l = __shfl_up(c4.w, 1), rt = __shfl_down(c4.x, 1);
            v[0] = lane == 0 ? le : l;
            v[1] = c4.x; v[2] = c4.y; v[3] = c4.z; v[4] = c4.w;
            v[5] = lane == 63 ? re : rt;
        };
        float up[6], md[6], dn[6];
        row6(rr, up);
        row6(rr + 1, md);
        row6(rr + 2, dn);
        float outs[4];
        uint32_t outd = 0;
        int cnt = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float c = md[e + 1];
            const bool det = c >= a.thr;
            const bool cand = det && c > up[e] && c > up[e + 1] && c > up[e + 2] && c > md[e] &&
                              c >= md[e + 2] && c >= dn[e] && c >= dn[e + 1] && c >= dn[e + 2];
            outs[e] = (c == -__builtin_inff()) ? 0.f : c;
            const uint32_t dv = (det ? ARGUS_DET : 0u) | (cand ? ARGUS_CAND : 0u);
            outd |= dv << (8 * e);
            cnt += (cand && x + e < a.W) ? 1 : 0;
        }
        const int64_t o = (int64_t)y * P + x;
        if (a.vec && x + 3 < a.W) {
            if (a.snr) *(float4 *)(a.snr + o) = make_float4(outs[0], outs[1], outs[2], outs[3]);
            *(uint32_t *)(a.det + o) = outd;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (x + e < a.W) {
                    if (a.snr) a.snr[o + e] = outs[e];
                    a.det[o + e] = (uint8_t)(outd >> (8 * e));
                }
            }
        }
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        if (lane == 0) a.counts[y * a.nsx + sx] = cnt;
    }
}

// Exclusive scan of one tile of STILE segment counts.
__global__ __launch_bounds__(NTHR) void scan_tiles_kernel(DetArgs a) {
    __shared__ int ws[NTHR / 64];
    const int t = blockIdx.x, tid = threadIdx.x;
    const int base = t * STILE + tid * (STILE / NTHR);
    int v[STILE / NTHR];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < STILE / NTHR; ++i) {
        int j = base + i;
        v[i] = j < a.nseg ? a.counts[j] : 0;
        sum += v[i];
    }
    // inclusive wave scan of the per-thread sums
    const int lane = tid & 63, w = tid >> 6;
    int inc = sum;
    for (int off = 1; off < 64; off <<= 1) {
        int n = __shfl_up(inc, off);
        if (lane >= off) inc += n;
    }
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    int wbase = 0;
    for (int i = 0; i < w; ++i) wbase += ws[i];
    int run = wbase + inc - sum;
#pragma unroll
    for (int i = 0; i < STILE / NTHR; ++i) {
        int j = base + i;
        if (j < a.nseg) a.local[j] = run;
        run += v[i];
    }
    if (tid == NTHR - 1) a.tile_sum[t] = wbase + inc;
}

template <bool SRC>
__global__ __launch_bounds__(NTHR) void detect_emit_kernel(DetArgs a) {
    const int lane = threadIdx.x & 63;
    // a wave reads the counts of 64 segments at once (one load per lane, most
    // segments hold no candidate) and visits those with candidates; groups of
    // 64 segments are strided over all waves
    const int nw = gridDim.x * (NTHR / 64);
    // the total goes out from the first wave (the sum of every scan tile)
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        int tot = 0;
        for (int t = lane; t < a.ntile; t += 64) tot += a.tile_sum[t];
        for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
        if (lane == 0) *a.n_cands = tot;
    }
    for (int s0 = (blockIdx.x * (NTHR / 64) + (threadIdx.x >> 6)) * 64; s0 < a.nseg; s0 += nw * 64) {
        const bool has = s0 + lane < a.nseg && a.counts[s0 + lane] != 0;
        uint64_t segs = __ballot(has);
        if (!segs) continue;
        // the 64 segments share one scan tile (STILE is a multiple of 64):
        // its offset is the sum of the tiles before it
        int toff = 0;
        for (int t = lane; t < s0 / STILE; t += 64) toff += a.tile_sum[t];
        for (int off = 32; off > 0; off >>= 1) toff += __shfl_xor(toff, off);
        while (segs) {
            const int seg = s0 + __builtin_ctzll(segs);
            segs &= segs - 1;
            int idx = toff + a.local[seg];
            const int y = seg / a.nsx, x0 = (seg % a.nsx) * SEG;
            const int64_t orow = (int64_t)y * a.pitch;
            const int K = 2 * a.r + 1;
            for (int c0 = 0; c0 < SEG && idx < a.cap; c0 += 64) {
                const int x = x0 + c0 + lane;
                const bool isc = x < a.W && (a.det[orow + x] & ARGUS_CAND);
                uint64_t bal = __ballot(isc);
                while (bal && idx < a.cap) {
                    const int l = __builtin_ctzll(bal);
                    bal &= bal - 1;
                    const int cx = x0 + c0 + l;
                    // PSF-weighted flux over unmasked in-image pixels of the window
                    double q = 0.0, f = 0.0;
                    for (int t = lane; t < K * K; t += 64) {
                        int xx = cx + t % K - a.r, yy = y + t / K - a.r;
                        if (xx < 0 || xx >= a.W || yy < 0 || yy >= a.H) continue;
                        int64_t o = (int64_t)yy * a.pitch + xx;
                        float V = a.dvar[o];
                        if (a.dmask[o] != 0 || !(V > 0.f)) continue;
                        double p = (double)a.psf[t];
                        q += p * p / (double)V;
                        f += p * (double)d_at<SRC>(a, o, xx, yy) / (double)V;
                    }
                    // source centroid: max(D, 0) over the unmasked in-image 3 x 3
                    double cs = 0.0, cxs = 0.0, cys = 0.0;
                    if constexpr (SRC) {
                        if (lane < 9) {
                            const int u = lane % 3 - 1, v = lane / 3 - 1, xx = cx + u, yy = y + v;
                            if (xx >= 0 && xx < a.W && yy >= 0 && yy < a.H) {
                                const int64_t o = (int64_t)yy * a.pitch + xx;
                                const float V = a.dvar[o];
                                if (a.dmask[o] == 0 && V > 0.f) {
                                    const double d = fmax((double)d_at<SRC>(a, o, xx, yy), 0.0);
                                    cs = d;
                                    cxs = u * d;
                                    cys = v * d;
                                }
                            }
                        }
                    }
                    for (int off = 32; off > 0; off >>= 1) {
                        q += __shfl_xor(q, off);
                        f += __shfl_xor(f, off);
                        if constexpr (SRC) {
                            cs += __shfl_xor(cs, off);
                            cxs += __shfl_xor(cxs, off);
                            cys += __shfl_xor(cys, off);
                        }
                    }
                    if (lane == 0) {
                        const float fl = q > 0.0 ? (float)(f / q) : __builtin_nanf("");
                        const float fe = q > 0.0 ? (float)(1.0 / sqrt(q)) : __builtin_nanf("");
                        if constexpr (SRC) {
                            argus_source c;
                            c.x = cx;
                            c.y = y;
                            c.xc = cs > 0.0 ? (float)(cx + cxs / cs) : __builtin_nanf("");
                            c.yc = cs > 0.0 ? (float)(y + cys / cs) : __builtin_nanf("");
                            c.snr = snr_at<SRC>(a, cx, y);
                            c.flux = fl;
                            c.flux_err = fe;
                            a.srcs[idx] = c;
                        } else {
                            argus_candidate c;
                            c.x = cx;
                            c.y = y;
                            c.snr = snr_at<SRC>(a, cx, y);
                            c.flux = fl;
                            c.flux_err = fe;
                            a.cands[idx] = c;
                        }
                    }
                    ++idx;
                }
            }
        }
    }
}

}  // namespace

namespace {

int launch_detect_any(argus_ctx *ctx, argus_dims d, const float *diff, const float *dvar,
                      const uint8_t *dmask, float thr, const float *psf, int r, float *snr,
                      uint8_t *det, argus_candidate *cands, argus_source *srcs, const float *grid,
                      int box, int32_t cap, int32_t *n_cands) {
    const bool src = grid != nullptr;
    DetArgs a;
    a.diff = diff; a.dvar = dvar; a.dmask = dmask; a.snr = snr; a.det = det;
    a.psf = psf; a.cands = cands; a.srcs = srcs; a.n_cands = n_cands;
    a.bg = src ? make_bg_grid(grid, box, d.width, d.height) : BgGrid{};
    a.pitch = d.pitch; a.W = d.width; a.H = d.height;
    a.nsx = (d.width + SEG - 1) / SEG;
    a.nseg = a.nsx * d.height;
    a.ntile = (a.nseg + STILE - 1) / STILE;
    a.r = r; a.cap = cap; a.thr = thr;
    auto al = [](const void *p, uintptr_t m) { return p == nullptr || ((uintptr_t)p % m) == 0; };
    a.vec = (d.pitch % 4 == 0) && al(diff, 16) && al(dvar, 16) && al(snr, 16) && al(dmask, 4) &&
            al(det, 4);
    size_t need = ((size_t)2 * a.nseg + a.ntile + 64) * sizeof(int32_t);
    int rc = argus_ws_reserve(ctx, need);
    if (rc) return rc;
    int32_t *w = (int32_t *)ctx->ws;
    a.counts = w;
    a.local = w + a.nseg;
    a.tile_sum = w + 2 * (size_t)a.nseg;
    argus_time_begin(ctx);
    const dim3 mg(a.nsx * ((d.height + ROWS - 1) / ROWS));
    if (src)
        hipLaunchKernelGGL(detect_map_kernel<true>, mg, dim3(NTHR), 0, ctx->stream, a);
    else
        hipLaunchKernelGGL(detect_map_kernel<false>, mg, dim3(NTHR), 0, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, src ? "source_map" : "detect_map");
    argus_time_begin(ctx);
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(a.ntile), dim3(NTHR), 0, ctx->stream, a);
    // one wave per 64 segments, at most enough to fill the device a few times over
    const int eblocks = std::max(1, std::min((a.nseg + 255) / 256, 8 * std::max(ctx->n_cu, 1)));
    if (src)
        hipLaunchKernelGGL(detect_emit_kernel<true>, dim3(eblocks), dim3(NTHR), 0, ctx->stream, a);
    else
        hipLaunchKernelGGL(detect_emit_kernel<false>, dim3(eblocks), dim3(NTHR), 0, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, src ? "source_emit" : "detect_emit");
    return ARGUS_OK;
}

}  // namespace

int launch_detect(argus_ctx *ctx, argus_dims d, const float *diff, const float *dvar,
                  const uint8_t *dmask, float thr, const float *psf, int r, float *snr,
                  uint8_t *det, argus_candidate *cands, int32_t cap, int32_t *n_cands) {
    return launch_detect_any(ctx, d, diff, dvar, dmask, thr, psf, r, snr, det, cands, nullptr,
                             nullptr, 0, cap, n_cands);
}

int launch_detect_sources(argus_ctx *ctx, argus_dims d, const float *cal, const float *var,
                          const uint8_t *mask, const float *grid, int box, float thr,
                          const float *psf, int r, float *snr, uint8_t *det, argus_source *srcs,
                          int32_t cap, int32_t *n_srcs) {
    return launch_detect_any(ctx, d, cal, var, mask, thr, psf, r, snr, det, nullptr, srcs, grid,
                             box, cap, n_srcs);
}
