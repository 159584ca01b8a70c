// Detection on the difference image: noise-normalised map, threshold,
// raster-ordered local maxima, stable compaction, PSF-weighted fluxes.
//
// detect_map: one workgroup per 1024-pixel row segment.  It forms the SNR of
//   the segment's row and its two neighbour rows (with a 1-pixel halo) in
//   LDS, writes snr and det_mask for its row and counts its candidates.
// detect_scan: exclusive scan of the segment counts (one workgroup) and the
//   list of segments that hold candidates.
// detect_emit: a wave per non-empty segment writes its candidates in raster
//   order at the scanned offsets and measures the PSF flux in FP64.
#include "internal.h"

namespace {

constexpr int SEG = 1024, NTHR = 256, PX = 4;

struct DetArgs {
    const float *diff, *dvar;
    const uint8_t *dmask;
    float *snr;
    uint8_t *det;
    int32_t *counts;           // [nseg]
    int32_t *offsets;          // [nseg]
    int32_t *nonempty;         // [nseg]
    int32_t *n_nonempty;       // [1]
    const float *psf;
    argus_candidate *cands;
    int32_t *n_cands;
    int64_t pitch;
    int W, H, nsx, nseg, r, cap;
    float thr;
};

__device__ __forceinline__ float snr_at(const DetArgs &a, int x, int y) {
    if (x < 0 || x >= a.W || y < 0 || y >= a.H) return -__builtin_inff();
    int64_t o = (int64_t)y * a.pitch + x;
    float V = a.dvar[o];
    if (a.dmask[o] != 0 || !(V > 0.f)) return 0.f;
    return a.diff[o] / __fsqrt_rn(V);
}

__global__ __launch_bounds__(NTHR) void detect_map_kernel(DetArgs a) {
    __shared__ float s[3][SEG + 2];
    __shared__ int red[NTHR / 64];
    const int sx = blockIdx.x, y = blockIdx.y, tid = threadIdx.x;
    const int x0 = sx * SEG;
    for (int i = tid; i < 3 * (SEG + 2); i += NTHR) {
        int row = i / (SEG + 2), c = i % (SEG + 2);
        int x = x0 - 1 + c;
        s[row][c] = (x <= x0 + SEG) ? snr_at(a, x, y - 1 + row) : -__builtin_inff();
    }
    __syncthreads();
    int cnt = 0;
    const int64_t orow = (int64_t)y * a.pitch;
#pragma unroll
    for (int j = 0; j < PX; ++j) {
        const int lx = tid * PX + j, x = x0 + lx;
        if (x >= a.W) break;
        const float c = s[1][lx + 1];
        const bool det = c >= a.thr;
        bool cand = det;
        // earlier neighbours (strictly greater), later neighbours (>=)
        cand = cand && c > s[0][lx] && c > s[0][lx + 1] && c > s[0][lx + 2] && c > s[1][lx];
        cand = cand && c >= s[1][lx + 2] && c >= s[2][lx] && c >= s[2][lx + 1] && c >= s[2][lx + 2];
        if (a.snr) a.snr[orow + x] = (c == -__builtin_inff()) ? 0.f : c;
        a.det[orow + x] = (det ? ARGUS_DET : 0u) | (cand ? ARGUS_CAND : 0u);
        cnt += cand;
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((tid & 63) == 0) red[tid >> 6] = cnt;
    __syncthreads();
    if (tid == 0) a.counts[y * a.nsx + sx] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(1024) void detect_scan_kernel(DetArgs a) {
    __shared__ int part[1024];
    __shared__ int npart[1024];
    const int tid = threadIdx.x, n = a.nseg;
    const int per = (n + 1023) / 1024;
    const int j0 = tid * per, j1 = min(j0 + per, n);
    int s = 0, ne = 0;
    for (int j = j0; j < j1; ++j) { s += a.counts[j]; ne += a.counts[j] > 0; }
    part[tid] = s;
    npart[tid] = ne;
    __syncthreads();
    // inclusive Hillis-Steele scans of the per-thread sums
    for (int off = 1; off < 1024; off <<= 1) {
        int v = tid >= off ? part[tid - off] : 0;
        int w = tid >= off ? npart[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        npart[tid] += w;
        __syncthreads();
    }
    int base = tid ? part[tid - 1] : 0;
    int nbase = tid ? npart[tid - 1] : 0;
    for (int j = j0; j < j1; ++j) {
        int c = a.counts[j];
        a.offsets[j] = base;
        base += c;
        if (c > 0) a.nonempty[nbase++] = j;
    }
    if (tid == 1023) {
        *a.n_cands = part[1023];
        *a.n_nonempty = npart[1023];
    }
}

__global__ __launch_bounds__(64) void detect_emit_kernel(DetArgs a) {
    const int lane = threadIdx.x;
    const int nne = *a.n_nonempty;
    for (int it = blockIdx.x; it < nne; it += gridDim.x) {
        const int seg = a.nonempty[it];
        const int y = seg / a.nsx, x0 = (seg % a.nsx) * SEG;
        int idx = a.offsets[seg];
        const int64_t orow = (int64_t)y * a.pitch;
        for (int c0 = 0; c0 < SEG && idx < a.cap; c0 += 64) {
            const int x = x0 + c0 + lane;
            const bool isc = x < a.W && (a.det[orow + x] & ARGUS_CAND);
            uint64_t bal = __ballot(isc);
            while (bal && idx < a.cap) {
                const int l = __builtin_ctzll(bal);
                bal &= bal - 1;
                const int cx = x0 + c0 + l;
                // PSF-weighted flux over unmasked in-image pixels of the window
                const int K = 2 * a.r + 1;
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
    a.r = r; a.cap = cap; a.thr = thr;
    size_t need = ((size_t)3 * a.nseg + 64) * sizeof(int32_t);
    int rc = argus_ws_reserve(ctx, need);
    if (rc) return rc;
    int32_t *w = (int32_t *)ctx->ws;
    a.counts = w;
    a.offsets = w + a.nseg;
    a.nonempty = w + 2 * (size_t)a.nseg;
    a.n_nonempty = w + 3 * (size_t)a.nseg;
    argus_time_begin(ctx);
    hipLaunchKernelGGL(detect_map_kernel, dim3(a.nsx, d.height), dim3(NTHR), 0, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "detect_map");
    hipLaunchKernelGGL(detect_scan_kernel, dim3(1), dim3(1024), 0, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    hipLaunchKernelGGL(detect_emit_kernel, dim3(1024), dim3(64), 0, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}
