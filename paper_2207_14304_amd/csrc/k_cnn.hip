// Learned kernel surrogate: stamp extraction, a 4-layer 3x3 CNN with BF16
// weights and activations and FP32 accumulation on MFMA, its backward pass,
// and Adam, all as HIP kernels.
//
// Network (per stamp pair, shared weights): four 'same' 3x3 convolutions
// (zero padding, cross-correlation) 2 -> 32 -> 32 -> 32 -> 32 with bias and
// ReLU; a spatial mean; a mean over the tile's valid stamps; a linear FP32
// head to the kernel coefficients.  Loss: mean squared error.
//
// Layouts: activations are channel-last [stamp][961][32] bf16 so that eight
// channels of one tap are one 16-byte LDS read; convolution weights are
// [out][tap][in] (k = tap*Cin + c), the FP32 master copy unpadded, the bf16
// copy padded to a multiple of 32 in k.  The backward-data pass is the same
// convolution with the weights transposed in (in, out) and flipped in taps.
#include <string.h>

#include <vector>

#include "internal.h"

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct argus_cnn {
    int C = 32, nout = 31, S = 64, r = 15, n = 31, npx = 961, max_tiles = 0;
    int cin[4] = {2, 32, 32, 32};
    int kp[4] = {32, 288, 288, 288};            // padded k per layer
    size_t w_off[4], b_off[4], hw_off, hb_off, P;
    float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    bf16 *wb[4] = {}, *wt[4] = {};             // forward and transposed-flipped copies
    bf16 *act[4] = {}, *dz[2] = {};            // activations, two dZ ping-pong buffers
    float *q = nullptr, *out = nullptr;         // per tile pooled features and outputs
    float *pool = nullptr, *dq = nullptr;       // per stamp pooled features, per tile dq
    float *part = nullptr;                      // gradient partials of layers 0..3 and the head
    size_t part_off[5] = {};                    // each block's region (floats from part)
    double *loss_part = nullptr;
    int32_t *order = nullptr, *nvalid = nullptr;   // the valid stamps' indices, their count
    int32_t *ticket = nullptr;                  // head workgroups done in a training step
    int step = 0;
    void *mem = nullptr;
};

namespace {

constexpr int NT = 256;

__device__ __forceinline__ float bf2f(bf16 x) { return (float)x; }

// ---------------------------------------------------------------------------
// Convolution: two workgroups per stamp, one per band of output rows (0..15
// and 16..30: 31 and 30 output tiles of 16 raster pixels x 32 channels
// spread over the waves); K = 9 * CIN (padded to 32) per tile.  A band holds
// its 18 input rows (with the halo) in LDS, so four workgroups fit a CU.  The
// weight fragments of every K step stay in registers (loaded once from global
// memory), so the tile loop reads only the activations from LDS.
// MODE 0: z + bias, ReLU.  MODE 1: gate by (g > 0) (backward data).
struct ConvArgs {
    const bf16 *in, *w, *gate;
    const float *bias;
    const int32_t *order, *nvalid;              // workgroup b < 2 *nvalid: stamp order[b / 2], band b % 2
    bf16 *out;
    float *pool;                                // forward: per stamp and band channel sums of out, or null
    int npx, n;                                 // pixels per stamp (961), stamps
};

template <int CIN>
struct ConvShape {
    static constexpr int KP = ((9 * CIN + 31) / 32) * 32, KS = KP / 32, PW = 33;
    static constexpr int BAND = 16, NBAND = 2;          // output rows per band, bands per stamp
    static constexpr int AROWS = BAND + 2;              // input rows y0 - 1 .. y0 + BAND
    static constexpr int ACT = (AROWS * PW * CIN + 7) & ~7;
};

// 4-wave workgroups, four per CU (LDS and registers)
template <int MODE>
constexpr int conv_threads() { return 256; }

template <int CIN, int MODE>
__global__ __launch_bounds__(conv_threads<MODE>(), 4) void cnn_conv_kernel(ConvArgs a) {
    constexpr int CTM = conv_threads<MODE>();
    using CS = ConvShape<CIN>;
    constexpr int KP = CS::KP, KS = CS::KS, W = 31, PW = CS::PW;
    extern __shared__ __align__(16) bf16 sm[];
    bf16 *act = sm;                             // [18][33][CIN]: rows y0 - 1 .. y0 + 16, zero border
    // the valid stamps come first in the grid (compacted order); the rest of
    // the workgroups leave at once
    if ((int)blockIdx.x >= *a.nvalid * CS::NBAND) return;
    const int s = a.order[blockIdx.x / CS::NBAND], tid = threadIdx.x;
    const int y0 = (blockIdx.x % CS::NBAND) * CS::BAND;          // first output row of the band
    const int p0 = y0 * W, p1 = min(a.npx, p0 + CS::BAND * W);   // its pixels
    const int lane = tid & 63, wave = tid >> 6, col = lane & 15, g = lane >> 4;
    // B fragments: output channels 2 col (B0) and 2 col + 1 (B1), k = ks*32 +
    // 8g .. +7, so a lane's two results of a pixel are adjacent channels
    bf16x8 B0[KS], B1[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        B0[ks] = *(const bf16x8 *)&a.w[(2 * col) * KP + ks * 32 + 8 * g];
        B1[ks] = *(const bf16x8 *)&a.w[(2 * col + 1) * KP + ks * 32 + 8 * g];
    }
    for (int i = tid; i < CS::ACT / 8; i += CTM) ((uint4 *)act)[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    // the input rows of the band that lie in the stamp: pixels q0 .. q1 - 1,
    // LDS row y - y0 + 1
    const int q0 = max(y0 - 1, 0) * W, q1 = min(a.npx, (y0 + CS::BAND + 1) * W);
    const bf16 *src = a.in + (size_t)s * a.npx * CIN;
    if constexpr (CIN % 8 == 0) {
        // 16-byte pieces (8 channels of a pixel), eight loads in flight per
        // thread before their LDS stores
        constexpr int C8 = CIN / 8, U = 8;
        const int n8 = (q1 - q0) * C8;
        const uint4 *src4 = (const uint4 *)(src + (size_t)q0 * CIN);
        for (int i0 = tid; i0 < n8; i0 += CTM * U) {
            uint4 v[U];
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const int i = i0 + e * CTM;
                v[e] = i < n8 ? src4[i] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const int i = i0 + e * CTM;
                if (i < n8) {
                    const int p = q0 + i / C8, c8 = i % C8, y = p / W, x = p % W;
                    *(uint4 *)&act[((y - y0 + 1) * PW + (x + 1)) * CIN + 8 * c8] = v[e];
                }
            }
        }
    } else {
        static_assert(CIN == 2, "the input layer has two channels");
        // one 4-byte word (both channels) per pixel, four loads in flight per
        // thread before their LDS stores
        constexpr int U = 4;
        const uint32_t *src2 = (const uint32_t *)src;
        for (int i0 = q0 + tid; i0 < q1; i0 += CTM * U) {
            uint32_t v[U];
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const int i = i0 + e * CTM;
                v[e] = i < q1 ? src2[i] : 0u;
            }
#pragma unroll
            for (int e = 0; e < U; ++e) {
                const int i = i0 + e * CTM;
                if (i < q1) {
                    const int y = i / W, x = i % W;
                    *(uint32_t *)&act[((y - y0 + 1) * PW + (x + 1)) * 2] = v[e];
                }
            }
        }
    }
    __syncthreads();
    bf16 *dst = a.out + (size_t)s * a.npx * 32;
    // A operand of tile t, step ks: pixel t*16 + col, inputs k = ks*32 + 8g .. +7
    auto load_a = [&](int t, int ks) -> bf16x8 {
        bf16x8 A;
        const int p = p0 + t * 16 + col, y = p / W - y0, x = p % W;
        const bool pin = p < p1;
        if constexpr (CIN == 32) {
            const int dy = ks / 3 - 1, dx = ks % 3 - 1;
            if (pin) {
                A = *(const bf16x8 *)&act[((y + 1 + dy) * PW + (x + 1 + dx)) * 32 + 8 * g];
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) A[e] = (bf16)0.f;
            }
        } else {
            // k = ks*32 + 8g + e is tap k / 2, channel k % 2: a lane's 8 values
            // are both channels of taps ks*16 + 4g .. +3, one 4-byte word each
#pragma unroll
            for (int e2 = 0; e2 < 4; ++e2) {
                const int tap = ks * 16 + 4 * g + e2;
                uint32_t w = 0u;
                if (pin && tap < 9) {
                    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
                    w = *(const uint32_t *)&act[((y + 1 + dy) * PW + (x + 1 + dx)) * 2];
                }
                A[2 * e2] = __builtin_bit_cast(bf16, (uint16_t)(w & 0xffffu));
                A[2 * e2 + 1] = __builtin_bit_cast(bf16, (uint16_t)(w >> 16));
            }
        }
        return A;
    };
    // the backward pass's gates (channels 2 col, 2 col + 1 of pixels 4g ..
    // 4g+3 of tile t), loaded before the tile's products so they are in flight
    auto load_gate = [&](int t, uint32_t (&gw)[4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pp = p0 + t * 16 + 4 * g + r;
            gw[r] = (MODE == 1 && pp < p1)
                        ? *(const uint32_t *)&a.gate[((size_t)s * a.npx + pp) * 32 + 2 * col]
                        : 0u;
        }
    };
    // pixels 4g .. 4g+3 of tile t, channels 2 col and 2 col + 1: one 4-byte
    // store per pixel
    float ps0 = 0.f, ps1 = 0.f;                 // channel sums of the stored outputs (forward)
    auto store = [&](int t, const floatx4 &r0, const floatx4 &r1, const uint32_t (&gw)[4]) {
        float b0 = 0.f, b1 = 0.f;
        if (MODE == 0) {
            b0 = a.bias[2 * col];
            b1 = a.bias[2 * col + 1];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pp = p0 + t * 16 + 4 * g + r;
            if (pp >= p1) continue;
            float v0 = r0[r], v1 = r1[r];
            if (MODE == 0) {
                v0 = fmaxf(v0 + b0, 0.f);
                v1 = fmaxf(v1 + b1, 0.f);
            } else {
                const bf16 *gv = (const bf16 *)&gw[r];
                v0 = bf2f(gv[0]) > 0.f ? v0 : 0.f;
                v1 = bf2f(gv[1]) > 0.f ? v1 : 0.f;
            }
            const bf16 o2[2] = {(bf16)v0, (bf16)v1};
            *(uint32_t *)&dst[(size_t)pp * 32 + 2 * col] = *(const uint32_t *)o2;
            if (MODE == 0) {
                ps0 += bf2f(o2[0]);
                ps1 += bf2f(o2[1]);
            }
        }
    };
    // two tiles per pass (t and t + NW): four independent accumulator chains
    constexpr int NW = CTM / 64;
    const int ntile = (p1 - p0 + 15) / 16;
    for (int t = wave; t < ntile; t += 2 * NW) {
        const bool two = t + NW < ntile;                // uniform across the wave
        uint32_t g0[4], g1[4];
        load_gate(t, g0);
        if (two) load_gate(t + NW, g1);
        floatx4 p0 = {0.f, 0.f, 0.f, 0.f}, p1 = p0, q0 = p0, q1 = p0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const bf16x8 A = load_a(t, ks);
            p0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B0[ks], p0, 0, 0, 0);
            p1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B1[ks], p1, 0, 0, 0);
            if (two) {
                const bf16x8 A2 = load_a(t + NW, ks);
                q0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2, B0[ks], q0, 0, 0, 0);
                q1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A2, B1[ks], q1, 0, 0, 0);
            }
        }
        store(t, p0, p1, g0);
        if (two) store(t + NW, q0, q1, g1);
    }
    if (MODE == 0 && a.pool) {
        // the spatial sum of the band (the head's pooling, fused): lanes col,
        // col + 16, col + 32, col + 48 hold the same two channels, then the
        // waves are added in order through LDS
        ps0 += __shfl_xor(ps0, 16);
        ps0 += __shfl_xor(ps0, 32);
        ps1 += __shfl_xor(ps1, 16);
        ps1 += __shfl_xor(ps1, 32);
        float *red = (float *)sm;               // [NW][32], after every wave is done with act
        __syncthreads();
        if (g == 0) {
            red[wave * 32 + 2 * col] = ps0;
            red[wave * 32 + 2 * col + 1] = ps1;
        }
        __syncthreads();
        if (tid < 32) {
            float sum = 0.f;
#pragma unroll
            for (int w = 0; w < NW; ++w) sum += red[w * 32 + tid];
            a.pool[((size_t)s * CS::NBAND + blockIdx.x % CS::NBAND) * 32 + tid] = sum;
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradients: dW[o][tap][c] = sum_p dZ[p][o] A_in[p + off(tap)][c] and
// db[o] = sum_p dZ[p][o] (one more MFMA tile whose B operand is all ones),
// summed over every valid stamp of the batch.  Workgroup b takes entries b,
// b + grid, ... of the compacted list of valid stamps, so the work is even
// whatever the tiles' fill; the per-workgroup partials are summed afterwards
// in a fixed order.  K steps are image rows (32 columns, the last one zero).
constexpr int WG_GROUPS = 16;   // weight-gradient workgroups per tile of the batch

struct WgradArgs {
    const bf16 *dz, *ain;
    const int32_t *order, *nvalid;              // the batch's valid stamps, their count
    float *part;                                // [workgroups][32 * 9 * CIN + 32]
    int npx;
};

// Weight gradients of a 32-channel layer, streamed in bands of R = 16 image
// rows so that a workgroup needs 78 KB of LDS and two fit a CU: while one
// stages a band from HBM the other runs its MFMAs.  Eight waves per
// workgroup; wave w < 6 owns the input row offset dy = w / 2 - 1 and the
// channel half w % 2 for all three horizontal taps and both halves of the
// output channels (6 accumulators): the two 16-byte reads of an input row
// segment give all three dx shifts in registers, so a band row costs a wave
// 4 LDS reads for 6 MFMAs.  Wave 6 takes the bias tile (B all ones), wave 7
// only stages.  Per stamp: bands y0 = 0 and 16 (15 rows, row 31 is zero).
struct Wg32 {
    static constexpr int R = 16, W = 31, NJ = 288;
    // channel strides padded to an odd number of 16-byte slots: the 16
    // channels a wave reads at once fall in distinct LDS banks
    static constexpr int DZS = R * 32 + 8;      // dZ [32 o][R rows][32 x], x = 31 is zero
    static constexpr int AR = R + 2, AW = 40;   // input rows y0 - 1 .. y0 + R, column x + 1
    static constexpr int AS = AR * AW + 8;
    static constexpr int NDZ = R * 16, NITEM = NDZ + AR * 16;   // pixel pairs per band
    static constexpr size_t bytes() { return ((size_t)32 * DZS + (size_t)32 * AS) * 2; }
};
constexpr int WT32 = 512;

__global__ __launch_bounds__(WT32, 4) void cnn_wgrad32_kernel(WgradArgs a) {
    using S = Wg32;
    constexpr int R = S::R, W = S::W, NJ = S::NJ, DZS = S::DZS, AW = S::AW, AS = S::AS;
    extern __shared__ __align__(16) bf16 sm[];
    bf16 *dzl = sm;
    bf16 *al = sm + 32 * DZS;
    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, g = lane >> 4;
    floatx4 acc[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // columns 32..39 of the input rows are read by the dx = +1 shifts of the
    // last segment and are never staged: zero them once
    for (int i = tid; i < (int)(S::bytes() / 16); i += WT32) ((uint4 *)sm)[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    const int dy = wave / 2 - 1, c = (wave & 1) * 16 + col;
    // a band item is a pair of horizontally adjacent pixels, all 32
    // channels (eight 16-byte loads); item q < NDZ is dZ row y0 + q / 16,
    // x = (2m, 2m+1), the rest input row y0 - 1 + r, x = (2m-1, 2m); pixels
    // outside the stamp read as zero
    auto load = [&](const bf16 *dzs, const bf16 *as, int y0, int q, uint4 (&v)[2][4]) {
        const bool isdz = q < S::NDZ;
        const int qq = isdz ? q : q - S::NDZ, m = qq % 16;
        const int y = isdz ? y0 + qq / 16 : y0 - 1 + qq / 16;
        const int x0 = isdz ? 2 * m : 2 * m - 1;
        const bf16 *base = isdz ? dzs : as;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int x = x0 + p;
            const bool in = y >= 0 && y < W && x >= 0 && x < W;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                v[p][k] = in ? ((const uint4 *)(base + (size_t)(y * W + x) * 32))[k] : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    auto store = [&](int q, const uint4 (&v)[2][4]) {
        const bool isdz = q < S::NDZ;
        const int qq = isdz ? q : q - S::NDZ, m = qq % 16, r = qq / 16;
        uint32_t *dst = isdz ? (uint32_t *)&dzl[r * 32 + 2 * m] : (uint32_t *)&al[r * AW + 2 * m];
        const int cs = (isdz ? DZS : AS) / 2;   // channel stride in words
#pragma unroll
        for (int o = 0; o < 32; ++o) {
            const uint32_t wa = (&v[0][o >> 3].x)[(o >> 1) & 3], wb = (&v[1][o >> 3].x)[(o >> 1) & 3];
            dst[o * cs] = (o & 1) ? ((wa >> 16) | (wb & 0xffff0000u)) : ((wa & 0xffffu) | (wb << 16));
        }
    };
    const int q1 = tid + WT32;
    const bool two = q1 < S::NITEM;
    const int nv = *a.nvalid;
    for (int k = b; k < nv; k += gridDim.x) {
        const int n = a.order[k];
        const bf16 *dzs = a.dz + (size_t)n * a.npx * 32;
        const bf16 *as = a.ain + (size_t)n * a.npx * 32;
        for (int y0 = 0; y0 < W; y0 += R) {
            {
                uint4 v0[2][4];
                load(dzs, as, y0, tid, v0);
                store(tid, v0);
            }
            if (two) {
                uint4 v1[2][4];
                load(dzs, as, y0, q1, v1);
                store(q1, v1);
            }
            __syncthreads();
            const int nr = min(R, W - y0);
            if (wave < 6) {
#pragma unroll 2
                for (int i = 0; i < nr; ++i) {
                    const bf16x8 A0 = *(const bf16x8 *)&dzl[col * DZS + i * 32 + 8 * g];
                    const bf16x8 A1 = *(const bf16x8 *)&dzl[(16 + col) * DZS + i * 32 + 8 * g];
                    const bf16 *rp = &al[c * AS + (i + 1 + dy) * AW + 8 * g];
                    const uint4 lo = *(const uint4 *)rp, hi = *(const uint4 *)(rp + 8);
                    uint4 s1, s2;
                    s1.x = __builtin_amdgcn_alignbyte(lo.y, lo.x, 2);
                    s1.y = __builtin_amdgcn_alignbyte(lo.z, lo.y, 2);
                    s1.z = __builtin_amdgcn_alignbyte(lo.w, lo.z, 2);
                    s1.w = __builtin_amdgcn_alignbyte(hi.x, lo.w, 2);
                    s2 = make_uint4(lo.y, lo.z, lo.w, hi.x);
                    const bf16x8 B0 = *(const bf16x8 *)&lo, B1 = *(const bf16x8 *)&s1,
                                 B2 = *(const bf16x8 *)&s2;
                    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B0, acc[0][0], 0, 0, 0);
                    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B0, acc[1][0], 0, 0, 0);
                    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B1, acc[0][1], 0, 0, 0);
                    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B1, acc[1][1], 0, 0, 0);
                    acc[0][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B2, acc[0][2], 0, 0, 0);
                    acc[1][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B2, acc[1][2], 0, 0, 0);
                }
            } else if (wave == 6) {
                // the bias tile: every column of B is one, so each column of
                // the product is db[o] = sum_p dZ[p][o]
                bf16x8 ones;
#pragma unroll
                for (int e = 0; e < 8; ++e) ones[e] = (bf16)1.f;
                for (int i = 0; i < nr; ++i) {
                    const bf16x8 A0 = *(const bf16x8 *)&dzl[col * DZS + i * 32 + 8 * g];
                    const bf16x8 A1 = *(const bf16x8 *)&dzl[(16 + col) * DZS + i * 32 + 8 * g];
                    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, ones, acc[0][0], 0, 0, 0);
                    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, ones, acc[1][0], 0, 0, 0);
                }
            }
            __syncthreads();
        }
    }
    // partials: dW[o][tap][c] at o * NJ + tap * 32 + c, tap = (dy + 1) * 3 + (dx + 1); db after
    float *part = a.part + (size_t)b * (32 * NJ + 32);
    if (wave < 6) {
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
            const int j = ((dy + 1) * 3 + dx) * 32 + c;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) part[(mt * 16 + 4 * g + r) * NJ + j] = acc[mt][dx][r];
        }
    } else if (wave == 6 && col == 0) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[32 * NJ + mt * 16 + 4 * g + r] = acc[mt][0][r];
    }
}

// Weight gradients of the first layer (2 input channels: 18 weight columns
// plus the bias), streamed in the same bands of 16 rows as the 32-channel
// kernel (36 KB of LDS, four workgroups per CU).  Wave 0 takes weight columns
// 0..15 (taps 0..7), wave 1 columns 16..17 (tap 8; the rest of its tile is
// zero), wave 2 the bias tile; every wave stages.  A column's tap and channel
// vary across the lanes, so each lane shifts its two 16-byte reads by its own
// dx.
struct Wg2 {
    static constexpr int R = 16, W = 31, CIN = 2, NJ = 9 * CIN;
    static constexpr int DZS = R * 32 + 8;      // dZ [32 o][R rows][32 x], as Wg32
    static constexpr int AR = R + 2, AW = 40;   // input rows y0 - 1 .. y0 + R, column x + 1
    static constexpr int AS = AR * AW + 8;
    static constexpr int NDZ = R * 16, NITEM = NDZ + AR * 16;   // pixel pairs per band
    static constexpr size_t bytes() { return ((size_t)32 * DZS + (size_t)CIN * AS) * 2; }
};

__global__ __launch_bounds__(WT32, 4) void cnn_wgrad2_kernel(WgradArgs a) {
    using S = Wg2;
    constexpr int R = S::R, W = S::W, NJ = S::NJ, DZS = S::DZS, AW = S::AW, AS = S::AS;
    extern __shared__ __align__(16) bf16 sm[];
    bf16 *dzl = sm;
    bf16 *al = sm + 32 * DZS;
    const int b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, g = lane >> 4;
    floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
    for (int i = tid; i < (int)(S::bytes() / 16); i += WT32) ((uint4 *)sm)[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    // this lane's weight column (waves 0 and 1): tap, channel, offsets
    const int j = wave * 16 + col;
    const bool jin = wave < 2 && j < NJ;
    const int tap = jin ? j / 2 : 0, cc = j % 2, dy = tap / 3 - 1, dx1 = tap % 3;   // dx1 = dx + 1
    // items as in the 32-channel kernel: q < NDZ a dZ pixel pair (all 32
    // channels), the rest an input pixel pair (x = 2m-1, 2m; one 4-byte word
    // of both channels each)
    auto load = [&](const bf16 *dzs, const bf16 *as, int y0, int q, uint4 (&v)[2][4]) {
        const bool isdz = q < S::NDZ;
        const int qq = isdz ? q : q - S::NDZ, m = qq % 16;
        const int y = isdz ? y0 + qq / 16 : y0 - 1 + qq / 16;
        const int x0 = isdz ? 2 * m : 2 * m - 1;
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int x = x0 + p;
            const bool in = y >= 0 && y < W && x >= 0 && x < W;
            if (isdz) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    v[p][k] = in ? ((const uint4 *)(dzs + (size_t)(y * W + x) * 32))[k] : make_uint4(0u, 0u, 0u, 0u);
            } else {
                v[p][0].x = in ? ((const uint32_t *)as)[y * W + x] : 0u;
            }
        }
    };
    auto store = [&](int q, const uint4 (&v)[2][4]) {
        const bool isdz = q < S::NDZ;
        const int qq = isdz ? q : q - S::NDZ, m = qq % 16, r = qq / 16;
        if (isdz) {
            uint32_t *dst = (uint32_t *)&dzl[r * 32 + 2 * m];
#pragma unroll
            for (int o = 0; o < 32; ++o) {
                const uint32_t wa = (&v[0][o >> 3].x)[(o >> 1) & 3], wb = (&v[1][o >> 3].x)[(o >> 1) & 3];
                dst[o * (DZS / 2)] = (o & 1) ? ((wa >> 16) | (wb & 0xffff0000u)) : ((wa & 0xffffu) | (wb << 16));
            }
        } else {
            uint32_t *dst = (uint32_t *)&al[r * AW + 2 * m];
            const uint32_t wa = v[0][0].x, wb = v[1][0].x;
            dst[0] = (wa & 0xffffu) | (wb << 16);                       // channel 0
            dst[AS / 2] = (wa >> 16) | (wb & 0xffff0000u);              // channel 1
        }
    };
    const int q1 = tid + WT32;
    const bool two = q1 < S::NITEM;
    const int nv = *a.nvalid;
    for (int k = b; k < nv; k += gridDim.x) {
        const int n = a.order[k];
        const bf16 *dzs = a.dz + (size_t)n * a.npx * 32;
        const bf16 *as = a.ain + (size_t)n * a.npx * 2;
        for (int y0 = 0; y0 < W; y0 += R) {
            {
                uint4 v0[2][4];
                load(dzs, as, y0, tid, v0);
                store(tid, v0);
            }
            if (two) {
                uint4 v1[2][4];
                load(dzs, as, y0, q1, v1);
                store(q1, v1);
            }
            __syncthreads();
            const int nr = min(R, W - y0);
            if (wave < 3) {
                for (int i = 0; i < nr; ++i) {
                    const bf16x8 A0 = *(const bf16x8 *)&dzl[col * DZS + i * 32 + 8 * g];
                    const bf16x8 A1 = *(const bf16x8 *)&dzl[(16 + col) * DZS + i * 32 + 8 * g];
                    bf16x8 B;
                    if (wave == 2) {
                        // the bias tile: every column of B is one
#pragma unroll
                        for (int e = 0; e < 8; ++e) B[e] = (bf16)1.f;
                    } else {
                        uint4 sel = make_uint4(0u, 0u, 0u, 0u);
                        if (jin) {
                            const bf16 *rp = &al[cc * AS + (i + 1 + dy) * AW + 8 * g];
                            const uint4 lo = *(const uint4 *)rp, hi = *(const uint4 *)(rp + 8);
                            uint4 s1;
                            s1.x = __builtin_amdgcn_alignbyte(lo.y, lo.x, 2);
                            s1.y = __builtin_amdgcn_alignbyte(lo.z, lo.y, 2);
                            s1.z = __builtin_amdgcn_alignbyte(lo.w, lo.z, 2);
                            s1.w = __builtin_amdgcn_alignbyte(hi.x, lo.w, 2);
                            const uint4 s2 = make_uint4(lo.y, lo.z, lo.w, hi.x);
                            sel = dx1 == 0 ? lo : (dx1 == 1 ? s1 : s2);
                        }
                        B = *(const bf16x8 *)&sel;
                    }
                    acc[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B, acc[0], 0, 0, 0);
                    acc[1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B, acc[1], 0, 0, 0);
                }
            }
            __syncthreads();
        }
    }
    // partials: dW[o][tap][c] at o * NJ + tap * 2 + c (= o * NJ + j); db after
    float *part = a.part + (size_t)b * (32 * NJ + 32);
    if (jin) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[(mt * 16 + 4 * g + r) * NJ + j] = acc[mt][r];
    } else if (wave == 2 && col == 0) {
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) part[32 * NJ + mt * 16 + 4 * g + r] = acc[mt][r];
    }
}

// ---------------------------------------------------------------------------
// Pooling (one workgroup per stamp) and head (one per tile).
struct HeadArgs {
    const bf16 *a4;
    const uint8_t *valid;
    const float *hw, *hb, *target;
    float *q, *out;
    bf16 *dz4;
    float *part;                                // head gradient partials [tiles][nout*32 + nout]
    double *loss_part;
    float *pool, *dq;                           // per stamp pooled features, per tile dq
    double *loss;                               // training: the batch loss
    int32_t *ticket;                            // training: workgroups done (zero between calls)
    int S, npx, nout, T;
};

// Per tile: mean of the pooled features over its valid stamps (the band
// sums of the last forward convolution / pixels), linear head.  Thread
// group k of 8 takes stamps k, k + 8, ...; the groups are added in order.
// TRAIN adds the head's backward pass in the same workgroup: the tile's
// loss, its head gradient partials and the gradient of the pooled features
// (already divided by valid stamps x pixels for the spread below); the last
// workgroup to finish sums the tiles' losses in tile order.
constexpr int HF_T = 256;
template <bool TRAIN>
__global__ __launch_bounds__(HF_T) void cnn_head_kernel(HeadArgs a) {
    __shared__ float qp[HF_T / 32][32];
    __shared__ int np[HF_T / 32];
    __shared__ float qs[32];
    __shared__ int s_nv;
    const int t = blockIdx.x, tid = threadIdx.x, c = tid & 31, grp = tid >> 5;
    float qsum = 0.f;
    int nv = 0;
    for (int s = grp; s < a.S; s += HF_T / 32) {
        const int n = t * a.S + s;
        if (!a.valid[n]) continue;
        ++nv;
        qsum += a.pool[(size_t)n * 64 + c] + a.pool[(size_t)n * 64 + 32 + c];
    }
    qp[grp][c] = qsum;
    if (c == 0) np[grp] = nv;
    __syncthreads();
    if (tid < 32) {
        float sum = 0.f;
        int n = 0;
#pragma unroll
        for (int k = 0; k < HF_T / 32; ++k) {
            sum += qp[k][tid];
            n += np[k];
        }
        qs[tid] = n > 0 ? sum / ((float)n * (float)a.npx) : 0.f;
        a.q[t * 32 + tid] = qs[tid];
        if (tid == 0) s_nv = n;
    }
    __syncthreads();
    float o = 0.f;
    if (tid < a.nout) {
        o = a.hb[tid];
        for (int k = 0; k < 32; ++k) o += a.hw[tid * 32 + k] * qs[k];
        a.out[t * a.nout + tid] = o;
    }
    if constexpr (TRAIN) {
        __shared__ float dout[64];
        __shared__ double lred[64];
        __shared__ int last;
        const float scale = 2.0f / (float)(a.T * a.nout);
        if (tid < 64) {
            double l = 0.0;
            float d = 0.f;
            if (tid < a.nout) {
                const float e = o - a.target[t * a.nout + tid];
                d = scale * e;
                l = (double)e * (double)e / (double)(a.T * a.nout);
            }
            dout[tid] = d;
            lred[tid] = l;
        }
        __syncthreads();
        float *part = a.part + (size_t)t * (a.nout * 32 + a.nout);
        for (int i = tid; i < a.nout * 32; i += HF_T) part[i] = dout[i / 32] * qs[i % 32];
        if (tid < a.nout) part[a.nout * 32 + tid] = dout[tid];
        if (tid < 32) {
            const int n = s_nv;
            const float inv = n > 0 ? 1.0f / ((float)n * (float)a.npx) : 0.f;
            float sd = 0.f;
            for (int j = 0; j < a.nout; ++j) sd += a.hw[j * 32 + tid] * dout[j];
            a.dq[t * 32 + tid] = sd * inv;
        }
        if (tid == 0) {
            double l = 0.0;
            for (int i = 0; i < 64; ++i) l += lred[i];
            a.loss_part[t] = l;
            __threadfence();                            // the loss part before the ticket
            last = atomicAdd(a.ticket, 1) == (int)gridDim.x - 1;
        }
        __syncthreads();
        if (last && tid == 0) {
            __threadfence();                            // every tile's part is visible
            double sum = 0.0;
            for (int i = 0; i < a.T; ++i) sum += ((volatile const double *)a.loss_part)[i];
            *a.loss = sum;
            *a.ticket = 0;                              // ready for the next step
        }
    }
}

// dZ of the last layer, DZ4_SPLIT items per valid stamp (compacted order),
// walked by a grid sized to the chip: the pooled-feature gradient gated by
// the ReLU of the forward activation, 8 channels per 16-byte load and store.
constexpr int DZ4_SPLIT = 4;
__device__ __forceinline__ void dz4_item(const HeadArgs &a, int n, int part, int tid) {
    const int t = n / a.S;
    const int g = tid & 3;                       // channels 8g .. 8g+7 (NT is a multiple of 4)
    float dq[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) dq[e] = a.dq[t * 32 + 8 * g + e];
    const uint4 *src = (const uint4 *)(a.a4 + (size_t)n * a.npx * 32);
    uint4 *dst = (uint4 *)(a.dz4 + (size_t)n * a.npx * 32);
    // whole pixels per part (four 16-byte pieces each), so piece i holds
    // channels 8 (i % 4) .. +7 = 8 g
    const int i0 = (part * a.npx / DZ4_SPLIT) * 4, i1 = ((part + 1) * a.npx / DZ4_SPLIT) * 4;
    for (int i = i0 + tid; i < i1; i += NT) {
        const uint4 v = src[i];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
        uint32_t o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float lo = __uint_as_float(w[e] << 16), hi = __uint_as_float(w[e] & 0xffff0000u);
            const bf16 blo = (bf16)(lo > 0.f ? dq[2 * e] : 0.f);
            const bf16 bhi = (bf16)(hi > 0.f ? dq[2 * e + 1] : 0.f);
            o[e] = (uint32_t)__builtin_bit_cast(uint16_t, blo) |
                   ((uint32_t)__builtin_bit_cast(uint16_t, bhi) << 16);
        }
        dst[i] = uint4{o[0], o[1], o[2], o[3]};
    }
}

__global__ __launch_bounds__(NT) void cnn_dz4_kernel(HeadArgs a, const int32_t *order,
                                                     const int32_t *nvalid) {
    const int nitems = *nvalid * DZ4_SPLIT, tid = threadIdx.x;
    for (int item = blockIdx.x; item < nitems; item += gridDim.x)
        dz4_item(a, order[item / DZ4_SPLIT], item % DZ4_SPLIT, tid);
}

// Indices of the valid stamps in increasing order and their count (one
// workgroup; a wave-level ballot scan per 1024-flag chunk).
constexpr int CMP_T = 1024;
__global__ __launch_bounds__(CMP_T) void cnn_compact_kernel(const uint8_t *valid, int n, int32_t *order,
                                                            int32_t *nvalid) {
    __shared__ int wsum[CMP_T / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int carry = 0;
    for (int base = 0; base < n; base += CMP_T) {
        const int i = base + tid;
        const bool v = i < n && valid[i] != 0;
        const uint64_t bal = __ballot(v);
        const int below = __builtin_popcountll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[w] = __builtin_popcountll(bal);
        __syncthreads();
        int off = carry;
        for (int q = 0; q < w; ++q) off += wsum[q];
        if (v) order[off + below] = i;
        int tot = 0;
        for (int q = 0; q < CMP_T / 64; ++q) tot += wsum[q];
        carry += tot;
        __syncthreads();
    }
    if (tid == 0) *nvalid = carry;
}

// Fixed-order sum of T per-tile partials into one gradient segment: a
// workgroup takes 32 consecutive entries; its 8 thread groups sum 8
// consecutive ranges of the partials (each in order, several loads in
// flight), then the 8 range sums are added in order.
constexpr int RED_W = 32, RED_G = 8;
struct ReduceArgs {
    const float *part[5];                       // per gradient block: [T][len] partials
    float *dst[5];
    int len[5], T[5];
};

// every gradient block of a step in one launch: blockIdx.y is the block
__global__ __launch_bounds__(RED_W * RED_G) void cnn_reduce_kernel(ReduceArgs ra) {
    __shared__ float rs[RED_G][RED_W];
    const int y = blockIdx.y;
    const float *part = ra.part[y];
    float *dst = ra.dst[y];
    const int len = ra.len[y], stride = len, T = ra.T[y];
    if ((int)blockIdx.x * RED_W >= len) return;     // uniform: this block is past the gradient
    const int j = threadIdx.x % RED_W, g = threadIdx.x / RED_W;
    const int i = blockIdx.x * RED_W + j;
    const int t0 = (int)((int64_t)g * T / RED_G), t1 = (int)((int64_t)(g + 1) * T / RED_G);
    float s = 0.f;
    if (i < len) {
        int t = t0;
        for (; t + 8 <= t1; t += 8) {
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = part[(size_t)(t + q) * stride + i];
#pragma unroll
            for (int q = 0; q < 8; ++q) s += v[q];
        }
        for (; t < t1; ++t) s += part[(size_t)t * stride + i];
    }
    rs[g][j] = s;
    __syncthreads();
    if (g == 0 && i < len) {
        float tot = 0.f;
#pragma unroll
        for (int q = 0; q < RED_G; ++q) tot += rs[q][j];
        dst[i] = tot;
    }
}

// Adam on every FP32 master weight, one thread per weight; a convolution
// weight's thread also writes its bf16 copies (forward [o][kp] and, above
// layer 0, transposed-flipped [c][(8 - tap) * 32 + o]), so the copies follow
// the update without another pass (the zero padding of the forward copy is
// written once, by cnn_pack).
struct AdamArgs {
    float *w, *m, *v;
    const float *g;
    size_t n;
    float lr, c1, c2;
    size_t w_off[4];
    int cin[4], kp[4];
    bf16 *wb[4], *wt[4];
};

__global__ void cnn_adam_kernel(AdamArgs a) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const float gi = a.g[i];
    const float mi = 0.9f * a.m[i] + 0.1f * gi;
    const float vi = 0.999f * a.v[i] + 0.001f * gi * gi;
    a.m[i] = mi;
    a.v[i] = vi;
    const float wi = a.w[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + 1e-8f);
    a.w[i] = wi;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        const size_t nl = (size_t)32 * 9 * a.cin[l];
        if (i >= a.w_off[l] && i < a.w_off[l] + nl) {
            const int j = (int)(i - a.w_off[l]), cin = a.cin[l];
            const int o = j / (9 * cin), k = j % (9 * cin), tap = k / cin, c = k % cin;
            a.wb[l][o * a.kp[l] + k] = (bf16)wi;
            if (a.wt[l]) a.wt[l][c * 288 + (8 - tap) * 32 + o] = (bf16)wi;
        }
    }
}

// bf16 copies of layer l: forward [o][kp] (zero padded) and, for the
// backward data pass, transposed-flipped [c][tap'*32 + o] = W[o][8 - tap'][c]
struct PackArgs {
    const float *w[4];
    bf16 *wb[4], *wt[4];                        // wt[0] is null (no data gradient below layer 0)
    int cin[4], kp[4];
};

// every layer in one launch: blockIdx.y is the layer
__global__ void cnn_pack_kernel(PackArgs pa) {
    const int l = blockIdx.y;
    const float *w = pa.w[l];
    const int cin = pa.cin[l], kp = pa.kp[l];
    bf16 *wb = pa.wb[l], *wt = pa.wt[l];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 32 * kp) {
        const int o = i / kp, k = i % kp;
        wb[i] = (bf16)(k < 9 * cin ? w[o * 9 * cin + k] : 0.f);
    }
    if (wt && i < 32 * 288) {
        const int c = i / 288, k = i % 288, tp = k / 32, o = k % 32;
        wt[i] = (bf16)w[(o * 9 + (8 - tp)) * cin + c];
    }
}

// ---------------------------------------------------------------------------
// Stamp extraction: one workgroup of NTS threads per tile.  Candidates are positive
// reference local maxima (strictly above earlier 8-neighbours in raster
// order, >= later ones) whose stamp lies inside the frame and whose peak
// stands snr_min noise sigmas above the tile's sky (the median of its
// unmasked reference pixels), ranked brightest first (raster order on ties).  Walking down the ranking, a candidate is
// kept when its stamp is unmasked in both frames and its peak stands
// snr_min noise sigmas above the reference stamp's border median; the walk
// stops at S kept.  Each kept stamp pair has its border medians removed and
// both are divided by the reference stamp's remaining sum and multiplied by
// STAMP_SCALE.
//
// The ranking holds at most MAXC candidates: a histogram of the candidates'
// float bit patterns (positive floats order like their bits; 4096 buckets
// of 1/8 octave) picks the lowest bucket whose suffix count fits, so every
// retained candidate is brighter than every dropped one.
constexpr int NTS = 1024;      // threads of the stamp extraction workgroup
constexpr int WW = 8;          // its waves that walk the ranking (LDS stamp slots)
constexpr int MAXC = 2048;
constexpr int NBUCKET = 4096;
// inputs near unit size: a unit-sum 31x31 stamp has values of order 1e-3,
// below what BF16 activations resolve next to biases of order 0.1
constexpr float STAMP_SCALE = 100.0f;

struct StampArgs {
    const float *ref, *rvar, *sci;
    const uint8_t *rmask, *smask;
    bf16 *X;                                    // [T][S][npx][2]
    uint8_t *valid;                             // [T][S]
    int32_t *overflow;
    int64_t pitch;
    int W, H, TX, TY, S, r;
    float snr_min;
};

// Border median of an n x n stamp (4(n-1) values) by a wave-wide bitonic
// sort in a 256-slot LDS buffer; the middle pair is averaged in FP32.
__device__ __forceinline__ float border_median_wave(const float *st, int n, float *buf, int lane) {
    const int nb = 4 * (n - 1);
    for (int i = lane; i < 256; i += 64) {
        float v = __builtin_inff();
        if (i < nb) {
            int y, x;
            if (i < n) { y = 0; x = i; }
            else if (i < 2 * n) { y = n - 1; x = i - n; }
            else if (i < 2 * n + n - 2) { y = 1 + (i - 2 * n); x = 0; }
            else { y = 1 + (i - 3 * n + 2); x = n - 1; }
            v = st[y * n + x];
        }
        buf[i] = v;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int k = 2; k <= 256; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = lane; i < 256; i += 64) {
                const int p = i ^ j;
                if (p > i) {
                    const bool up = (i & k) == 0;
                    const float a = buf[i], b = buf[p];
                    if ((a > b) == up) { buf[i] = b; buf[p] = a; }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    const float med = (nb & 1) ? buf[nb / 2] : (buf[nb / 2 - 1] + buf[nb / 2]) * 0.5f;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return med;
}

// Order-preserving unsigned key of a float (NaN excluded by the caller).
__device__ __forceinline__ uint32_t fkey(float v) {
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unkey(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Key of the rank-k (0-based) unmasked reference value of the tile: radix
// select over 8-bit digits with a 256-bin LDS histogram per pass.
__device__ uint32_t tile_select(const StampArgs &a, int x0, int y0, int tw, int npix, int k,
                                int *bins) {
    const int tid = threadIdx.x;
    const int64_t P = a.pitch;
    uint32_t prefix = 0, pmask = 0;
    __shared__ int s_digit, s_k;
    if (tid == 0) s_k = k;
    for (int shift = 24; shift >= 0; shift -= 8) {
        if (tid < 256) bins[tid] = 0;
        __syncthreads();
        for (int i = tid; i < npix; i += NTS) {
            const int64_t o = (int64_t)(y0 + i / tw) * P + x0 + i % tw;
            if (a.rmask[o] != 0) continue;
            const uint32_t key = fkey(a.ref[o]);
            if ((key & pmask) == prefix) atomicAdd(&bins[(key >> shift) & 255u], 1);
        }
        __syncthreads();
        if (tid == 0) {
            int kk = s_k, d = 0;
            while (d < 255 && kk >= bins[d]) { kk -= bins[d]; ++d; }
            s_digit = d;
            s_k = kk;
        }
        __syncthreads();
        prefix |= (uint32_t)s_digit << shift;
        pmask |= 255u << shift;
        __syncthreads();
    }
    return prefix;
}

__global__ __launch_bounds__(NTS) void stamps_kernel(StampArgs a) {
    __shared__ unsigned long long keys[MAXC];
    __shared__ int hist[NBUCKET];
    __shared__ int psum[NTS];
    __shared__ int ncand, nacc, cutoff, dropped;
    __shared__ int flag[WW];
    __shared__ float fmed[WW];
    __shared__ int acc_y[64], acc_x[64];
    __shared__ float acc_m[64];
    extern __shared__ __align__(16) float sst[];   // per walking wave: 2 stamps + 256 sort slots
    const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tx = t % a.TX, ty = t / a.TX;
    const int x0 = (int)((int64_t)tx * a.W / a.TX), x1 = (int)((int64_t)(tx + 1) * a.W / a.TX);
    const int y0 = (int)((int64_t)ty * a.H / a.TY), y1 = (int)((int64_t)(ty + 1) * a.H / a.TY);
    const int r = a.r, n = 2 * r + 1, npx = n * n;
    const int64_t P = a.pitch;
    const int tw = x1 - x0, npix = tw * (y1 - y0);
    // the tile's sky: median of its unmasked reference pixels (middle pair
    // averaged in FP32); +inf when every pixel is masked (no candidates)
    __shared__ int s_nun;
    if (tid == 0) s_nun = 0;
    __syncthreads();
    {
        int cnt = 0;
        for (int i = tid; i < npix; i += NTS)
            cnt += a.rmask[(int64_t)(y0 + i / tw) * P + x0 + i % tw] == 0;
        atomicAdd(&s_nun, cnt);
    }
    __syncthreads();
    const int nun = s_nun;
    float sky = __builtin_inff();
    if (nun > 0) {
        const float v1 = unkey(tile_select(a, x0, y0, tw, npix, (nun - 1) / 2, hist));
        if (nun & 1) {
            sky = v1;
        } else {
            const float v2 = unkey(tile_select(a, x0, y0, tw, npix, nun / 2, hist));
            sky = (v1 + v2) * 0.5f;
        }
    }
    for (int i = tid; i < NBUCKET; i += NTS) hist[i] = 0;
    if (tid == 0) { ncand = 0; nacc = 0; }
    __syncthreads();
    // candidate test; the stamp-in-frame bound keeps every neighbour in the frame
    auto is_cand = [&](int y, int x, float &c) -> bool {
        if (y < r || x < r || y >= a.H - r || x >= a.W - r) return false;
        const int64_t o = (int64_t)y * P + x;
        const float *q = a.ref + o;
        c = q[0];
        if (!(c > 0.f)) return false;
        if (!(c > q[-P - 1] && c > q[-P] && c > q[-P + 1] && c > q[-1] && c >= q[1] &&
              c >= q[P - 1] && c >= q[P] && c >= q[P + 1]))
            return false;
        const float vv = a.rvar[o];
        return vv > 0.f && (c - sky) / sqrtf(vv) >= a.snr_min;
    };
    for (int i = tid; i < npix; i += NTS) {
        float c;
        if (is_cand(y0 + i / tw, x0 + i % tw, c)) atomicAdd(&hist[__float_as_uint(c) >> 20], 1);
    }
    __syncthreads();
    // lowest bucket whose suffix count fits in MAXC
    {
        int sum = 0;
        for (int b = 0; b < NBUCKET / NTS; ++b) sum += hist[tid * (NBUCKET / NTS) + b];
        psum[tid] = sum;
    }
    __syncthreads();
    if (tid == 0) {
        constexpr int CH = NBUCKET / NTS;
        int tot = 0;
        for (int i = 0; i < NTS; ++i) tot += psum[i];
        int acc = 0, cut = NBUCKET;                 // buckets >= cut are kept
        int i = NTS - 1;
        while (i >= 0 && acc + psum[i] <= MAXC) {   // whole chunks from the top
            acc += psum[i];
            cut = i * CH;
            --i;
        }
        if (i >= 0) {                               // then single buckets
            for (int b = i * CH + CH - 1; b >= i * CH; --b) {
                if (acc + hist[b] > MAXC) break;
                acc += hist[b];
                cut = b;
            }
        }
        cutoff = cut;
        dropped = tot - acc;
    }
    __syncthreads();
    for (int i = tid; i < npix; i += NTS) {
        const int y = y0 + i / tw, x = x0 + i % tw;
        float c;
        if (is_cand(y, x, c) && (int)(__float_as_uint(c) >> 20) >= cutoff) {
            const int slot = atomicAdd(&ncand, 1);
            // brightest first, raster index breaking ties (c > 0)
            keys[slot] = ((unsigned long long)(0xFFFFFFFFu - __float_as_uint(c)) << 32) |
                         (unsigned int)((int64_t)y * a.W + x);
        }
    }
    __syncthreads();
    const int nc = ncand;
    int m2 = 1;
    while (m2 < nc) m2 <<= 1;
    for (int i = nc + tid; i < m2; i += NTS) keys[i] = ~0ull;
    __syncthreads();
    for (int k = 2; k <= m2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < m2; i += NTS) {
                const int p = i ^ j;
                if (p > i) {
                    const bool up = (i & k) == 0;
                    const unsigned long long u = keys[i], w = keys[p];
                    if ((u > w) == up) { keys[i] = w; keys[p] = u; }
                }
            }
            __syncthreads();
        }
    }
    // walk the ranking WW candidates at a time, one per walking wave
    float *ws = sst + (size_t)(wave < WW ? wave : 0) * (2 * npx + 256);
    for (int k0 = 0; k0 < nc; k0 += WW) {
        if (nacc >= a.S) break;                 // uniform: shared, read after a barrier
        const int k = k0 + wave;
        int ok = 0;
        float med = 0.f;
        if (wave < WW && k < nc) {
            const unsigned int idx = (unsigned int)(keys[k] & 0xFFFFFFFFull);
            const int y = idx / a.W, x = idx % a.W;
            int bad = 0;
            for (int i = lane; i < npx; i += 64) {
                const int64_t o = (int64_t)(y - r + i / n) * P + (x - r + i % n);
                bad |= a.rmask[o] | a.smask[o];
                ws[i] = a.ref[o];
            }
            if (!__any(bad)) {
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
                med = border_median_wave(ws, n, ws + 2 * npx, lane);
                const int64_t o = (int64_t)y * P + x;
                const float v = a.ref[o], vv = a.rvar[o];
                ok = vv > 0.f && (v - med) / sqrtf(vv) >= a.snr_min;
            }
        }
        if (lane == 0 && wave < WW) { flag[wave] = ok; fmed[wave] = med; }
        __syncthreads();
        if (tid == 0) {
            for (int w = 0; w < WW && nacc < a.S; ++w) {
                if (!flag[w]) continue;
                const unsigned int idx = (unsigned int)(keys[k0 + w] & 0xFFFFFFFFull);
                acc_y[nacc] = idx / a.W;
                acc_x[nacc] = idx % a.W;
                acc_m[nacc] = fmed[w];
                ++nacc;
            }
        }
        __syncthreads();
    }
    if (tid == 0 && nacc < a.S && dropped > 0) atomicAdd(a.overflow, 1);
    // stamps: one walking wave per kept stamp
    for (int s = wave; s < a.S && wave < WW; s += WW) {
        const int64_t base = ((int64_t)t * a.S + s) * npx * 2;
        uint8_t ok = 0;
        if (s < nacc) {
            const int y = acc_y[s], x = acc_x[s];
            for (int i = lane; i < npx; i += 64) {
                const int64_t o = (int64_t)(y - r + i / n) * P + (x - r + i % n);
                ws[i] = a.ref[o];
                ws[npx + i] = a.sci[o];
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const float mr = acc_m[s];
            const float ms = border_median_wave(ws + npx, n, ws + 2 * npx, lane);
            float sum = 0.f;
            for (int i = lane; i < npx; i += 64) sum += ws[i] - mr;
            for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
            if (sum > 0.f) {
                const float inv = STAMP_SCALE / sum;
                for (int i = lane; i < npx; i += 64) {
                    a.X[base + 2 * i] = (bf16)((ws[i] - mr) * inv);
                    a.X[base + 2 * i + 1] = (bf16)((ws[npx + i] - ms) * inv);
                }
                ok = 1;
            }
        }
        if (!ok)
            for (int i = lane; i < 2 * npx; i += 64) a.X[base + i] = (bf16)0.f;
        if (lane == 0) a.valid[t * a.S + s] = ok;
    }
}

template <int CIN, int MODE>
int conv_launch(argus_ctx *ctx, const ConvArgs &ca) {
    size_t lds = (size_t)ConvShape<CIN>::ACT * sizeof(bf16);
    ARGUS_HIP_CHECK(ctx, hipFuncSetAttribute((const void *)cnn_conv_kernel<CIN, MODE>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL((cnn_conv_kernel<CIN, MODE>), dim3(ca.n * ConvShape<CIN>::NBAND),
                       dim3(conv_threads<MODE>()), lds,
                       ctx->stream, ca);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

int wgrad2_launch(argus_ctx *ctx, const WgradArgs &wa, int T) {
    size_t lds = Wg2::bytes();
    ARGUS_HIP_CHECK(ctx, hipFuncSetAttribute((const void *)cnn_wgrad2_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(cnn_wgrad2_kernel, dim3(T * WG_GROUPS), dim3(WT32), lds, ctx->stream, wa);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

int wgrad32_launch(argus_ctx *ctx, const WgradArgs &wa, int T) {
    size_t lds = Wg32::bytes();
    ARGUS_HIP_CHECK(ctx, hipFuncSetAttribute((const void *)cnn_wgrad32_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(cnn_wgrad32_kernel, dim3(T * WG_GROUPS), dim3(WT32), lds, ctx->stream, wa);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

int cnn_pack(argus_ctx *ctx, argus_cnn *c) {
    PackArgs pa;
    for (int l = 0; l < 4; ++l) {
        pa.w[l] = c->master + c->w_off[l];
        pa.wb[l] = c->wb[l];
        pa.wt[l] = l > 0 ? c->wt[l] : nullptr;
        pa.cin[l] = c->cin[l];
        pa.kp[l] = c->kp[l];
    }
    hipLaunchKernelGGL(cnn_pack_kernel, dim3((32 * 288 + 255) / 256, 4), dim3(256), 0, ctx->stream, pa);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

// forward over T tiles of S stamps; activations stay for the backward pass
// the head (forward only) is left to the caller when head is false: the
// training step runs it fused with its backward pass
int cnn_forward_impl(argus_ctx *ctx, argus_cnn *c, const bf16 *X, const uint8_t *valid, int T,
                     bool head = true) {
    hipLaunchKernelGGL(cnn_compact_kernel, dim3(1), dim3(CMP_T), 0, ctx->stream, valid, T * c->S,
                       c->order, c->nvalid);
    ConvArgs ca;
    ca.npx = c->npx;
    ca.n = T * c->S;
    ca.order = c->order;
    ca.nvalid = c->nvalid;
    ca.gate = nullptr;
    for (int l = 0; l < 4; ++l) {
        ca.in = l == 0 ? X : c->act[l - 1];
        ca.w = c->wb[l];
        ca.bias = c->master + c->b_off[l];
        ca.out = c->act[l];
        ca.pool = l == 3 ? c->pool : nullptr;
        int rc = l == 0 ? conv_launch<2, 0>(ctx, ca) : conv_launch<32, 0>(ctx, ca);
        if (rc) return rc;
    }
    HeadArgs ha;
    ha.a4 = c->act[3]; ha.valid = valid; ha.hw = c->master + c->hw_off; ha.hb = c->master + c->hb_off;
    ha.target = nullptr; ha.q = c->q; ha.out = c->out; ha.dz4 = nullptr; ha.part = nullptr;
    ha.loss_part = nullptr; ha.S = c->S; ha.npx = c->npx; ha.nout = c->nout; ha.T = T;
    ha.pool = c->pool; ha.dq = c->dq; ha.loss = nullptr; ha.ticket = nullptr;
    if (head) hipLaunchKernelGGL(cnn_head_kernel<false>, dim3(T), dim3(HF_T), 0, ctx->stream, ha);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

// CNN outputs -> coefficient vectors [n][nb + 1] with a zero background
__global__ void sur_coeffs_kernel(const float *out, int n, int nb, double *coeffs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * (nb + 1)) return;
    const int s = i / (nb + 1), k = i % (nb + 1);
    coeffs[i] = k < nb ? (double)out[s * nb + k] : 0.0;
}

// Per solve: weighted least-squares background given the surrogate kernel,
// its chi^2 and the acceptance test against the plain fit.
struct SelectArgs {
    const double *sur, *chi2_0, *swd, *sw, *plain, *plain_chi2;
    const int64_t *n0, *plain_n;
    double ref_chi2_dof, factor;
    double *out, *chi2_dof;
    int32_t *accepted;
    int n, nb, n_unknowns;
};

__global__ void sur_select_kernel(SelectArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n) return;
    const double sw = a.sw[s], swd = a.swd[s];
    const int64_t n0 = a.n0[s];
    double b = 0.0, chi2s = a.chi2_0[s];
    if (sw > 0.0) {
        b = swd / sw;
        chi2s -= swd * swd / sw;
    }
    const double rs = n0 > 1 ? chi2s / (double)(n0 - 1) : __builtin_inf();
    double rp = a.ref_chi2_dof;
    if (a.plain_chi2) {
        const int64_t dp = a.plain_n[s] - a.n_unknowns;
        rp = dp > 0 ? a.plain_chi2[s] / (double)dp : __builtin_inf();
    }
    const bool acc = rs <= a.factor * rp;
    const int nc = a.nb + 1;
    for (int k = 0; k < nc; ++k) {
        double v;
        if (acc) v = k < a.nb ? a.sur[s * nc + k] : b;
        else v = a.plain ? a.plain[s * nc + k] : __builtin_nan("");
        a.out[s * nc + k] = v;
    }
    a.chi2_dof[s] = rs;
    a.accepted[s] = acc ? 1 : 0;
}

}  // namespace

extern "C" {

int argus_surrogate_coeffs(argus_ctx *ctx, int n_solves, int n_basis, const float *cnn_out,
                           double *coeffs) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    if (!cnn_out || !coeffs) return argus_fail(ctx, ARGUS_EINVAL, "argus_surrogate_coeffs: null pointer");
    if (n_solves < 1 || n_basis < 1 || n_basis > 64)
        return argus_fail(ctx, ARGUS_ESHAPE, "n_solves >= 1, n_basis 1..64");
    const int tot = n_solves * (n_basis + 1);
    hipLaunchKernelGGL(sur_coeffs_kernel, dim3((tot + 255) / 256), dim3(256), 0, ctx->stream,
                       cnn_out, n_solves, n_basis, coeffs);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

int argus_surrogate_select(argus_ctx *ctx, int n_solves, int n_basis, const double *sur_coeffs,
                           const double *chi2_0, const int64_t *n_0, const double *sum_wd,
                           const double *sum_w, const double *plain_coeffs,
                           const double *plain_chi2, const int64_t *plain_n,
                           double ref_chi2_dof, double factor, double *coeffs_out,
                           double *chi2_dof, int32_t *accepted) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    if (!sur_coeffs || !chi2_0 || !n_0 || !sum_wd || !sum_w || !coeffs_out || !chi2_dof || !accepted)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_surrogate_select: null pointer");
    if (n_solves < 1 || n_basis < 1 || n_basis > 64)
        return argus_fail(ctx, ARGUS_ESHAPE, "n_solves >= 1, n_basis 1..64");
    if ((plain_chi2 == nullptr) != (plain_n == nullptr))
        return argus_fail(ctx, ARGUS_EINVAL, "plain_chi2 and plain_n go together");
    if (!plain_chi2 && !(ref_chi2_dof > 0.0))
        return argus_fail(ctx, ARGUS_EINVAL, "without plain chi^2 a reference chi^2/dof > 0 is needed");
    if (!(factor > 0.0)) return argus_fail(ctx, ARGUS_EINVAL, "factor must be > 0");
    SelectArgs a;
    a.sur = sur_coeffs; a.chi2_0 = chi2_0; a.swd = sum_wd; a.sw = sum_w; a.plain = plain_coeffs;
    a.plain_chi2 = plain_chi2; a.n0 = n_0; a.plain_n = plain_n; a.ref_chi2_dof = ref_chi2_dof;
    a.factor = factor; a.out = coeffs_out; a.chi2_dof = chi2_dof; a.accepted = accepted;
    a.n = n_solves; a.nb = n_basis; a.n_unknowns = n_basis + 1;
    hipLaunchKernelGGL(sur_select_kernel, dim3((n_solves + 63) / 64), dim3(64), 0, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

int argus_cnn_create(argus_ctx *ctx, int max_tiles, argus_cnn **out) {
    if (!ctx || !out || max_tiles < 1 || max_tiles > 65536) return ARGUS_EINVAL;
    *out = nullptr;
    argus_cnn *c = new argus_cnn();
    c->max_tiles = max_tiles;
    size_t off = 0;
    for (int l = 0; l < 4; ++l) {
        c->w_off[l] = off;
        off += (size_t)32 * 9 * c->cin[l];
        c->b_off[l] = off;
        off += 32;
    }
    c->hw_off = off;
    off += (size_t)c->nout * 32;
    c->hb_off = off;
    off += c->nout;
    c->P = off;
    const size_t N = (size_t)max_tiles * c->S, A = N * c->npx * 32;
    const size_t head_stride = (size_t)c->nout * 32 + c->nout;
    size_t bytes = 4 * c->P * sizeof(float);                        // master, grad, m, v
    bytes += 4 * 32 * 288 * sizeof(bf16) * 2;                       // wb, wt
    bytes += (4 * A + 2 * A) * sizeof(bf16);                        // act, dz
    bytes += (size_t)max_tiles * (32 + c->nout) * sizeof(float);    // q, out
    size_t part_len = 0;                        // per workgroup (layers) or tile (head) partials
    for (int l = 0; l < 5; ++l) {
        c->part_off[l] = part_len;
        part_len += l < 4 ? (size_t)max_tiles * WG_GROUPS * (32 * 9 * c->cin[l] + 32)
                          : (size_t)max_tiles * head_stride;
    }
    bytes += part_len * sizeof(float);
    bytes += (size_t)max_tiles * sizeof(double) + 4096;
    bytes += (2 * N + max_tiles) * 32 * sizeof(float) + 512;        // pool (two bands), dq
    bytes += N * sizeof(int32_t) + 512;                              // order, nvalid
    bytes += 32 * 256;                                               // 256-byte alignment of each region
    if (hipMalloc(&c->mem, bytes) != hipSuccess) {
        delete c;
        return argus_fail(ctx, ARGUS_ENOMEM, "cnn buffers (%zu bytes)", bytes);
    }
    char *p = (char *)c->mem;
    auto take = [&](size_t b) { char *q = p; p += (b + 255) & ~(size_t)255; return (void *)q; };
    c->master = (float *)take(c->P * 4);
    c->grad = (float *)take(c->P * 4);
    c->m = (float *)take(c->P * 4);
    c->v = (float *)take(c->P * 4);
    for (int l = 0; l < 4; ++l) {
        c->wb[l] = (bf16 *)take(32 * 288 * 2);
        c->wt[l] = (bf16 *)take(32 * 288 * 2);
    }
    for (int l = 0; l < 4; ++l) c->act[l] = (bf16 *)take(A * 2);
    for (int l = 0; l < 2; ++l) c->dz[l] = (bf16 *)take(A * 2);
    c->q = (float *)take((size_t)max_tiles * 32 * 4);
    c->out = (float *)take((size_t)max_tiles * c->nout * 4);
    c->part = (float *)take(part_len * 4);
    c->loss_part = (double *)take((size_t)max_tiles * 8);
    c->pool = (float *)take(N * 64 * 4);
    c->dq = (float *)take((size_t)max_tiles * 32 * 4);
    c->order = (int32_t *)take(N * 4);
    c->nvalid = (int32_t *)take(64);
    c->ticket = (int32_t *)take(64);
    if (hipMemsetAsync(c->mem, 0, 4 * c->P * sizeof(float) + 1024, ctx->stream) != hipSuccess ||
        hipMemsetAsync(c->ticket, 0, 64, ctx->stream) != hipSuccess) {
        (void)hipFree(c->mem);
        delete c;
        return argus_fail(ctx, ARGUS_EHIP, "cnn init");
    }
    *out = c;
    return ARGUS_OK;
}

void argus_cnn_destroy(argus_cnn *c) {
    if (!c) return;
    if (c->mem) (void)hipFree(c->mem);
    delete c;
}

int argus_cnn_n_params(const argus_cnn *c) { return c ? (int)c->P : -1; }

int argus_cnn_set_weights(argus_ctx *ctx, argus_cnn *c, const float *host) {
    if (!ctx || !c || !host) return ARGUS_EINVAL;
    ARGUS_HIP_CHECK(ctx, hipMemcpyAsync(c->master, host, c->P * 4, hipMemcpyHostToDevice, ctx->stream));
    ARGUS_HIP_CHECK(ctx, hipMemsetAsync(c->m, 0, c->P * 4, ctx->stream));
    ARGUS_HIP_CHECK(ctx, hipMemsetAsync(c->v, 0, c->P * 4, ctx->stream));
    ARGUS_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    c->step = 0;
    return cnn_pack(ctx, c);
}

int argus_cnn_get_weights(argus_ctx *ctx, argus_cnn *c, float *host) {
    if (!ctx || !c || !host) return ARGUS_EINVAL;
    ARGUS_HIP_CHECK(ctx, hipMemcpyAsync(host, c->master, c->P * 4, hipMemcpyDeviceToHost, ctx->stream));
    ARGUS_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    return ARGUS_OK;
}

int argus_cnn_get_grads(argus_ctx *ctx, argus_cnn *c, float *host) {
    if (!ctx || !c || !host) return ARGUS_EINVAL;
    ARGUS_HIP_CHECK(ctx, hipMemcpyAsync(host, c->grad, c->P * 4, hipMemcpyDeviceToHost, ctx->stream));
    ARGUS_HIP_CHECK(ctx, hipStreamSynchronize(ctx->stream));
    return ARGUS_OK;
}

int argus_cnn_forward(argus_ctx *ctx, argus_cnn *c, const uint16_t *X, const uint8_t *valid, int T,
                      float *out) {
    if (!ctx || !c || !X || !valid || !out) return ARGUS_EINVAL;
    ctx->err.clear();
    if ((uintptr_t)X % 4) return argus_fail(ctx, ARGUS_EINVAL, "stamps X must be 4-byte aligned");
    if (T < 1 || T > c->max_tiles) return argus_fail(ctx, ARGUS_ESHAPE, "T %d not in 1..%d", T, c->max_tiles);
    int rc = cnn_forward_impl(ctx, c, (const bf16 *)X, valid, T);
    if (rc) return rc;
    ARGUS_HIP_CHECK(ctx, hipMemcpyAsync(out, c->out, (size_t)T * c->nout * 4, hipMemcpyDeviceToDevice,
                                        ctx->stream));
    return ARGUS_OK;
}

int argus_cnn_train_step(argus_ctx *ctx, argus_cnn *c, const uint16_t *X, const uint8_t *valid,
                         const float *target, int T, float lr, double *loss) {
    if (!ctx || !c || !X || !valid || !target || !loss) return ARGUS_EINVAL;
    ctx->err.clear();
    if ((uintptr_t)X % 4) return argus_fail(ctx, ARGUS_EINVAL, "stamps X must be 4-byte aligned");
    if (T < 1 || T > c->max_tiles) return argus_fail(ctx, ARGUS_ESHAPE, "T %d not in 1..%d", T, c->max_tiles);
    if (!(lr >= 0.f)) return argus_fail(ctx, ARGUS_EINVAL, "learning rate must be >= 0");
    const bf16 *Xb = (const bf16 *)X;
    int rc = cnn_forward_impl(ctx, c, Xb, valid, T, false);
    if (rc) return rc;
    // head forward and backward, the loss -> dZ of layer 3 (in dz[1])
    HeadArgs ha;
    ha.a4 = c->act[3]; ha.valid = valid; ha.hw = c->master + c->hw_off; ha.hb = c->master + c->hb_off;
    ha.target = target; ha.q = c->q; ha.out = c->out; ha.dz4 = c->dz[1];
    ha.part = c->part + c->part_off[4];
    ha.loss_part = c->loss_part; ha.S = c->S; ha.npx = c->npx; ha.nout = c->nout; ha.T = T;
    ha.pool = c->pool; ha.dq = c->dq; ha.loss = loss; ha.ticket = c->ticket;
    hipLaunchKernelGGL(cnn_head_kernel<true>, dim3(T), dim3(HF_T), 0, ctx->stream, ha);
    const int dz4_grid = std::max(1, std::min(T * c->S * DZ4_SPLIT, 8 * std::max(ctx->n_cu, 1)));
    hipLaunchKernelGGL(cnn_dz4_kernel, dim3(dz4_grid), dim3(NT), 0, ctx->stream, ha,
                       (const int32_t *)c->order, (const int32_t *)c->nvalid);
    // every gradient block is summed by one launch after the last weight gradients
    ReduceArgs ra;
    ra.part[4] = ha.part;
    ra.dst[4] = c->grad + c->hw_off;
    ra.len[4] = c->nout * 32 + c->nout;
    ra.T[4] = T;
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    // conv layers 3..0: weight gradients, then dZ of the layer below
    int cur = 1;
    for (int l = 3; l >= 0; --l) {
        WgradArgs wa;
        wa.dz = c->dz[cur];
        wa.ain = l == 0 ? Xb : c->act[l - 1];
        wa.order = c->order;                         // compacted by this step's forward pass
        wa.nvalid = c->nvalid;
        wa.part = c->part + c->part_off[l];
        wa.npx = c->npx;
        rc = l == 0 ? wgrad2_launch(ctx, wa, T) : wgrad32_launch(ctx, wa, T);
        if (rc) return rc;
        ra.part[l] = wa.part;
        ra.dst[l] = c->grad + c->w_off[l];
        ra.len[l] = 32 * 9 * c->cin[l] + 32;
        ra.T[l] = T * WG_GROUPS;
        if (l > 0) {
            ConvArgs ca;
            ca.in = c->dz[cur];
            ca.w = c->wt[l];
            ca.gate = c->act[l - 1];
            ca.bias = nullptr;
            ca.pool = nullptr;
            ca.order = c->order;                     // compacted by this step's forward pass
            ca.nvalid = c->nvalid;
            ca.out = c->dz[cur ^ 1];
            ca.npx = c->npx;
            ca.n = T * c->S;
            if ((rc = conv_launch<32, 1>(ctx, ca))) return rc;
            cur ^= 1;
        }
    }
    int rx = 0;
    for (int k = 0; k < 5; ++k) rx = ra.len[k] > rx ? ra.len[k] : rx;
    hipLaunchKernelGGL(cnn_reduce_kernel, dim3((rx + RED_W - 1) / RED_W, 5), dim3(RED_W * RED_G), 0,
                       ctx->stream, ra);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    // Adam on the FP32 master weights and their bf16 copies
    c->step += 1;
    const float c1 = 1.0f - powf(0.9f, (float)c->step), c2 = 1.0f - powf(0.999f, (float)c->step);
    AdamArgs aa;
    aa.w = c->master; aa.m = c->m; aa.v = c->v; aa.g = c->grad; aa.n = c->P;
    aa.lr = lr; aa.c1 = c1; aa.c2 = c2;
    for (int l = 0; l < 4; ++l) {
        aa.w_off[l] = c->w_off[l];
        aa.cin[l] = c->cin[l];
        aa.kp[l] = c->kp[l];
        aa.wb[l] = c->wb[l];
        aa.wt[l] = l > 0 ? c->wt[l] : nullptr;
    }
    hipLaunchKernelGGL(cnn_adam_kernel, dim3((unsigned)((c->P + 255) / 256)), dim3(256), 0,
                       ctx->stream, aa);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

int argus_extract_stamps(argus_ctx *ctx, argus_dims d, const float *ref, const float *ref_var,
                         const uint8_t *ref_mask, const float *sci, const uint8_t *sci_mask,
                         int tiles_x, int tiles_y, float snr_min, int stamps_per_tile,
                         int half, uint16_t *X, uint8_t *valid, int32_t *overflow) {
    if (!ctx) return ARGUS_EINVAL;
    ctx->err.clear();
    if (d.width < 1 || d.height < 1 || d.pitch < d.width)
        return argus_fail(ctx, ARGUS_ESHAPE, "bad dims");
    if (!ref || !ref_var || !ref_mask || !sci || !sci_mask || !X || !valid || !overflow)
        return argus_fail(ctx, ARGUS_EINVAL, "argus_extract_stamps: null pointer");
    if (tiles_x < 1 || tiles_y < 1 || stamps_per_tile < 1 || stamps_per_tile > 64 || half < 1 ||
        half > 15)
        return argus_fail(ctx, ARGUS_ESHAPE, "tiles >= 1, 1..64 stamps, half width 1..15");
    if (tiles_x > d.width || tiles_y > d.height)
        return argus_fail(ctx, ARGUS_ESHAPE, "more tiles than pixels");
    if (!(snr_min > 0.f))
        return argus_fail(ctx, ARGUS_EINVAL, "snr_min must be > 0");
    if ((int64_t)d.width * d.height >= ((int64_t)1 << 32))
        return argus_fail(ctx, ARGUS_ESHAPE, "frame too large for 32-bit pixel keys");
    StampArgs a;
    a.ref = ref; a.rvar = ref_var; a.sci = sci; a.rmask = ref_mask; a.smask = sci_mask;
    a.X = (bf16 *)X; a.valid = valid; a.overflow = overflow;
    a.pitch = d.pitch; a.W = d.width; a.H = d.height; a.TX = tiles_x; a.TY = tiles_y;
    a.S = stamps_per_tile; a.r = half; a.snr_min = snr_min;
    const int npx = (2 * half + 1) * (2 * half + 1);
    size_t lds = (size_t)WW * (2 * npx + 256) * sizeof(float);
    ARGUS_HIP_CHECK(ctx, hipFuncSetAttribute((const void *)stamps_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(stamps_kernel, dim3(tiles_x * tiles_y), dim3(NTS), lds, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

}  // extern "C"
