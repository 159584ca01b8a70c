// Median-filtered background map of a calibrated frame.
//
// bg_cell: one workgroup per box x box cell (box <= 64, so a thread holds at
//   most 16 pixels in registers).  The cell's level is the exact median of
//   its unmasked values: a 4-pass radix select on order-preserving 32-bit keys
//   of the FP32 values (8 bits per pass, LDS histogram, one wave scans it),
//   and for an even count the next key by a count and a minimum; the mean of
//   the middle pair is formed in FP64 and rounded once.
// bg_filter: one thread per cell, median of the present levels of its 3 x 3
//   neighbourhood (insertion sort of at most 9 values).
// bg_map: bilinear interpolation between cell centres to every pixel (only
//   when the caller asks for the full-resolution map; detection evaluates the
//   same interpolation on the fly).
#include "internal.h"
#include "background.h"

namespace {

constexpr int NTHR = 256, MAXV = 16;     // 16 x 256 = 4096 = 64 x 64 pixels

__device__ __forceinline__ uint32_t f2key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key2f(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

struct CellArgs {
    const float *cal;
    const uint8_t *mask;
    float *levels;
    int64_t pitch;
    int W, H, box, gx, gy;
};

__device__ int block_sum_i(int v, int *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int s = 0;
    for (int i = 0; i < NTHR / 64; ++i) s += red[i];
    return s;
}

__global__ __launch_bounds__(NTHR) void bg_cell_kernel(CellArgs a) {
    __shared__ int hist[256];
    __shared__ int red[NTHR / 64];
    __shared__ uint32_t sel[2];          // selected prefix, remaining rank
    __shared__ uint32_t kmin;
    const int tid = threadIdx.x;
    const int ci = blockIdx.x % a.gx, cj = blockIdx.x / a.gx;
    const int x0 = ci * a.box, y0 = cj * a.box;
    const int cw = min(a.box, a.W - x0), ch = min(a.box, a.H - y0);
    const int np = cw * ch;
    uint32_t key[MAXV];
    int nv = 0;
    // every load of a thread is issued before any is used
    float v[MAXV];
    uint8_t m[MAXV];
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
        const int i = tid + k * NTHR;
        const int ii = i < np ? i : 0;
        const int64_t o = (int64_t)(y0 + ii / cw) * a.pitch + x0 + ii % cw;
        v[k] = a.cal[o];
        m[k] = a.mask[o];
    }
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
        const int i = tid + k * NTHR;
        const bool ok = i < np && m[k] == 0;
        key[k] = ok ? f2key(v[k]) : 0u;      // 0 never equals a selected prefix with ok = false
        nv += ok ? 1 : 0;
    }
    uint32_t okbits = 0;
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
        const int i = tid + k * NTHR;
        if (i < np && m[k] == 0) okbits |= 1u << k;
    }
    const int n = block_sum_i(nv, red);
    if (n == 0) {
        if (tid == 0) a.levels[blockIdx.x] = __builtin_nanf("");
        return;
    }
    // k-th smallest key (0-based): the lower middle for an even count
    const uint32_t k1 = (uint32_t)((n - 1) / 2);
    if (tid == 0) { sel[0] = 0u; sel[1] = k1; }
    uint32_t pmask = 0u;
    for (int shift = 24; shift >= 0; shift -= 8) {
        hist[tid] = 0;
        __syncthreads();
        const uint32_t prefix = sel[0];
#pragma unroll
        for (int k = 0; k < MAXV; ++k)
            if (((okbits >> k) & 1u) && (key[k] & pmask) == prefix)
                atomicAdd(&hist[(key[k] >> shift) & 255u], 1);
        __syncthreads();
        if (tid < 64) {
            // lane l owns bins 4l .. 4l+3; inclusive scan of the lane sums
            const int h0 = hist[4 * tid], h1 = hist[4 * tid + 1], h2 = hist[4 * tid + 2],
                      h3 = hist[4 * tid + 3];
            const int s = h0 + h1 + h2 + h3;
            int inc = s;
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(inc, off);
                if (tid >= off) inc += t;
            }
            const uint32_t r = sel[1];
            const int before = inc - s;
            if ((uint32_t)before <= r && r < (uint32_t)inc) {
                // the rank falls in this lane's four bins
                int acc = before, d = 4 * tid;
                const int hh[4] = {h0, h1, h2, h3};
                for (int q = 0; q < 4; ++q) {
                    if (r < (uint32_t)(acc + hh[q])) { d = 4 * tid + q; break; }
                    acc += hh[q];
                }
                sel[0] = prefix | ((uint32_t)d << shift);
                sel[1] = r - (uint32_t)acc;
            }
        }
        pmask |= 255u << shift;
        __syncthreads();
    }
    const uint32_t kk1 = sel[0];
    float med;
    if (n & 1) {
        med = key2f(kk1);
    } else {
        // upper middle: the same key if it repeats past rank k1, else the
        // smallest key above it
        int le = 0;
#pragma unroll
        for (int k = 0; k < MAXV; ++k) le += (((okbits >> k) & 1u) && key[k] <= kk1) ? 1 : 0;
        if (tid == 0) kmin = 0xffffffffu;
        const int nle = block_sum_i(le, red);
        uint32_t kk2 = kk1;
        if ((uint32_t)nle < k1 + 2u) {
            uint32_t mn = 0xffffffffu;
#pragma unroll
            for (int k = 0; k < MAXV; ++k)
                if (((okbits >> k) & 1u) && key[k] > kk1 && key[k] < mn) mn = key[k];
            for (int off = 32; off > 0; off >>= 1) {
                const uint32_t t = (uint32_t)__shfl_xor((int)mn, off);
                mn = t < mn ? t : mn;
            }
            if ((tid & 63) == 0) atomicMin(&kmin, mn);
            __syncthreads();
            kk2 = kmin;
        }
        med = (float)(0.5 * ((double)key2f(kk1) + (double)key2f(kk2)));
    }
    if (tid == 0) a.levels[blockIdx.x] = med;
}

__global__ void bg_filter_kernel(const float *levels, float *grid, int gx, int gy) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= gx * gy) return;
    const int i = c % gx, j = c / gx;
    float v[9];
    int n = 0;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
            const int ii = i + di, jj = j + dj;
            if (ii < 0 || ii >= gx || jj < 0 || jj >= gy) continue;
            const float l = levels[jj * gx + ii];
            if (l != l) continue;                           // no level
            int p = n++;
            while (p > 0 && v[p - 1] > l) { v[p] = v[p - 1]; --p; }
            v[p] = l;
        }
    float out = 0.f;
    if (n & 1) out = v[n / 2];
    else if (n > 0) out = (float)(0.5 * ((double)v[n / 2 - 1] + (double)v[n / 2]));
    grid[c] = out;
}

__global__ __launch_bounds__(NTHR) void bg_map_kernel(BgGrid g, float *map, int64_t pitch, int W,
                                                      int H) {
    const int x = blockIdx.x * NTHR + threadIdx.x, y = blockIdx.y;
    if (x >= W) return;
    map[(int64_t)y * pitch + x] = bg_at(g, x, y);
}

}  // namespace

int launch_background(argus_ctx *ctx, argus_dims d, const float *cal, const uint8_t *mask, int box,
                      float *levels, float *grid, float *map) {
    const int gx = (d.width + box - 1) / box, gy = (d.height + box - 1) / box;
    float *lev = levels;
    if (!lev) {
        int rc = argus_ws_reserve(ctx, (size_t)gx * gy * sizeof(float) + 256);
        if (rc) return rc;
        lev = (float *)ctx->ws;
    }
    CellArgs a{cal, mask, lev, d.pitch, d.width, d.height, box, gx, gy};
    argus_time_begin(ctx);
    hipLaunchKernelGGL(bg_cell_kernel, dim3(gx * gy), dim3(NTHR), 0, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    hipLaunchKernelGGL(bg_filter_kernel, dim3((gx * gy + 255) / 256), dim3(256), 0, ctx->stream,
                       (const float *)lev, grid, gx, gy);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "background");
    if (map) {
        BgGrid g = make_bg_grid(grid, box, d.width, d.height);
        argus_time_begin(ctx);
        hipLaunchKernelGGL(bg_map_kernel, dim3((d.width + NTHR - 1) / NTHR, d.height), dim3(NTHR), 0,
                           ctx->stream, g, map, d.pitch, d.width, d.height);
        ARGUS_HIP_CHECK(ctx, hipGetLastError());
        argus_time_end(ctx, "background_map");
    }
    return ARGUS_OK;
}
