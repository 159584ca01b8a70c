// Detection on the difference image: noise-normalised map, threshold,
// raster-ordered local maxima, stable compaction, PSF-weighted fluxes.
//
// detect_map: one workgroup per 1024 x 4 tile.  It forms the SNR of its rows
//   and one halo row/column on each side in LDS, writes snr and det_mask and
//   counts the candidates of each 1024-pixel row segment.
// scan_tiles / scan_top: exclusive scan of the segment counts (1024-count
//   tiles in parallel, then the tile totals) -> raster-order offsets.
// detect_emit: one wave per segment with candidates writes them in raster
//   order at their offsets and measures the PSF flux in FP64.
#include "internal.h"

namespace {

constexpr int SEG = 1024, ROWS = 4, NTHR = 256, PXT = SEG / 64;   // 16 px per thread
constexpr int STILE = 1024;                                        // counts per scan tile

struct DetArgs {
    const float *diff, *dvar;
    const uint8_t *dmask;
    float *snr;
    uint8_t *det;
    int32_t *counts;           // [nseg]   candidates per row segment
    int32_t *local;            // [nseg]   offset within its scan tile
    int32_t *tile_sum;         // [ntile]
    int32_t *tile_off;         // [ntile]
    const float *psf;
    argus_candidate *cands;
    int32_t *n_cands;
    int64_t pitch;
    int W, H, nsx, nseg, ntile, r, cap;
    float thr;
};

// SNR of one pixel: D / sqrt(V) where the pixel is unmasked and V > 0, else 0;
// off-image pixels are -inf for the neighbour comparisons.
__device__ __forceinline__ float snr_at(const DetArgs &a, int x, int y) {
    if (x < 0 || x >= a.W || y < 0 || y >= a.H) return -__builtin_inff();
    int64_t o = (int64_t)y * a.pitch + x;
    float V = a.dvar[o];
    if (a.dmask[o] != 0 || !(V > 0.f)) return 0.f;
    return a.diff[o] * __builtin_amdgcn_rsqf(V);
}

__global__ __launch_bounds__(NTHR) void detect_map_kernel(DetArgs a) {
    __shared__ float s[ROWS + 2][SEG + 4];
    const int sx = blockIdx.x, y0 = blockIdx.y * ROWS, tid = threadIdx.x;
    const int x0 = sx * SEG;
    for (int i = tid; i < (ROWS + 2) * (SEG + 2); i += NTHR) {
        int row = i / (SEG + 2), c = i % (SEG + 2);
        s[row][c] = snr_at(a, x0 - 1 + c, y0 - 1 + row);
    }
    __syncthreads();
    const int rr = tid >> 6, lane = tid & 63;     // wave rr owns tile row rr
    const int y = y0 + rr;
    int cnt = 0;
    if (y < a.H) {
        // pixel lx = 64 j + lane: consecutive lanes read consecutive LDS words
        const int64_t orow = (int64_t)y * a.pitch;
#pragma unroll 4
        for (int j = 0; j < PXT; ++j) {
            const int lx = 64 * j + lane, x = x0 + lx;
            const float c = s[rr + 1][lx + 1];
            const bool det = c >= a.thr;
            bool cand = det && c > s[rr][lx] && c > s[rr][lx + 1] && c > s[rr][lx + 2] &&
                        c > s[rr + 1][lx];
            cand = cand && c >= s[rr + 1][lx + 2] && c >= s[rr + 2][lx] &&
                   c >= s[rr + 2][lx + 1] && c >= s[rr + 2][lx + 2];
            if (x < a.W) {
                if (a.snr) a.snr[orow + x] = (c == -__builtin_inff()) ? 0.f : c;
                a.det[orow + x] = (det ? ARGUS_DET : 0u) | (cand ? ARGUS_CAND : 0u);
                cnt += cand ? 1 : 0;
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if (lane == 0 && y < a.H) a.counts[y * a.nsx + sx] = cnt;
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

__global__ __launch_bounds__(64) void scan_top_kernel(DetArgs a) {
    const int lane = threadIdx.x;
    int carry = 0;
    for (int b = 0; b < a.ntile; b += 64) {
        const int j = b + lane;
        const int v = j < a.ntile ? a.tile_sum[j] : 0;
        int inc = v;
        for (int off = 1; off < 64; off <<= 1) {
            int n = __shfl_up(inc, off);
            if (lane >= off) inc += n;
        }
        if (j < a.ntile) a.tile_off[j] = carry + inc - v;
        carry += __shfl(inc, 63);
    }
    if (lane == 0) *a.n_cands = carry;
}

__global__ __launch_bounds__(NTHR) void detect_emit_kernel(DetArgs a) {
    const int lane = threadIdx.x & 63;
    const int seg = blockIdx.x * (NTHR / 64) + (threadIdx.x >> 6);
    if (seg >= a.nseg || a.counts[seg] == 0) return;
    int idx = a.tile_off[seg / STILE] + a.local[seg];
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
                f += p * (double)a.diff[o] / (double)V;
            }
            for (int off = 32; off > 0; off >>= 1) {
                q += __shfl_xor(q, off);
                f += __shfl_xor(f, off);
            }
            if (lane == 0) {
                argus_candidate c;
                c.x = cx;
                c.y = y;
                c.snr = snr_at(a, cx, y);
                c.flux = q > 0.0 ? (float)(f / q) : __builtin_nanf("");
                c.flux_err = q > 0.0 ? (float)(1.0 / sqrt(q)) : __builtin_nanf("");
                a.cands[idx] = c;
            }
            ++idx;
        }
    }
}

}  // namespace

int launch_detect(argus_ctx *ctx, argus_dims d, const float *diff, const float *dvar,
                  const uint8_t *dmask, float thr, const float *psf, int r, float *snr,
                  uint8_t *det, argus_candidate *cands, int32_t cap, int32_t *n_cands) {
    DetArgs a;
    a.diff = diff; a.dvar = dvar; a.dmask = dmask; a.snr = snr; a.det = det;
    a.psf = psf; a.cands = cands; a.n_cands = n_cands;
    a.pitch = d.pitch; a.W = d.width; a.H = d.height;
    a.nsx = (d.width + SEG - 1) / SEG;
    a.nseg = a.nsx * d.height;
    a.ntile = (a.nseg + STILE - 1) / STILE;
    a.r = r; a.cap = cap; a.thr = thr;
    size_t need = ((size_t)2 * a.nseg + 2 * a.ntile + 64) * sizeof(int32_t);
    int rc = argus_ws_reserve(ctx, need);
    if (rc) return rc;
    int32_t *w = (int32_t *)ctx->ws;
    a.counts = w;
    a.local = w + a.nseg;
    a.tile_sum = w + 2 * (size_t)a.nseg;
    a.tile_off = a.tile_sum + a.ntile;
    argus_time_begin(ctx);
    hipLaunchKernelGGL(detect_map_kernel, dim3(a.nsx, (d.height + ROWS - 1) / ROWS), dim3(NTHR), 0,
                       ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "detect_map");
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(a.ntile), dim3(NTHR), 0, ctx->stream, a);
    hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(64), 0, ctx->stream, a);
    hipLaunchKernelGGL(detect_emit_kernel, dim3((a.nseg + 3) / 4), dim3(NTHR), 0, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}
