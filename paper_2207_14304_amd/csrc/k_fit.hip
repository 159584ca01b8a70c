// Kernel fit: basis tables, fused basis convolution + normal-equation
// accumulation on MFMA, FP64 reduction of the partial sums, and the
// Jacobi-scaled FP64 Cholesky solve.
//
// Model (Alard & Lupton 1998; Alard 2000): the design row of pixel p is
//   X_p = [P_m(p) C_k(p)]_{k<nb, m<nP} ++ [P_m(p)]_{m<nPbg},
// with C_k = ref (x) B_k.  Every entry of A = sum w X X^T is a moment
//   G_{ab}[k][l] = sum_p w_p xt^a yt^b c_k(p) c_l(p),   a+b <= 2D,
// of the 32-vector c = (C_0..C_{nb-1}, 1, 0...) (the 1 carries the
// background), and b = sum w X S needs R_{ab}[k] = sum w xt^a yt^b c_k S,
// a+b <= D.  Along one image row yt is constant, so a workgroup accumulates
// only the xt-moments of the row on MFMA (FP32, 64 pixels) and then adds
// yt^b times them into FP64 running sums: 2D+1 Gram blocks per pixel instead
// of (2D+1)(2D+2)/2.
#include "fit_accum.h"

using argus_fit::FitArgs;
using argus_fit::FitShape;
using argus_fit::SW;
using argus_fit::NTHR;
using argus_fit::qidx;

namespace {

// ---------------------------------------------------------------------------
// Basis tables, computed on the device in FP64 from the spec.
// B_k(u,v) = exp(-(u^2+v^2)/2s^2) u^i v^j; B_0 -> unit sum; k>=1 with i, j
// even -> B_k - (sum B_k) B_0; k >= 1 -> unit L2 norm.  In separable form
// B'_k = alpha_k f_{g,i}(u) f_{g,j}(v) + beta_k B_0raw.
__global__ void basis_tables_kernel(argus_kernel_spec s, BasisTables *T) {
    __shared__ int kg[32], ki[32], kj[32], kp[32];
    __shared__ double alpha[32], beta[32];
    __shared__ double S0;
    const int h = s.half_width, K = 2 * h + 1;
    if (threadIdx.x == 0) {
        int k = 0, p = 0;
        for (int g = 0; g < s.n_gauss; ++g)
            for (int i = 0; i <= s.degree[g]; ++i, ++p)
                for (int j = 0; j <= s.degree[g] - i; ++j, ++k) {
                    kg[k] = g; ki[k] = i; kj[k] = j; kp[k] = p;
                }
        T->nb = k;
        T->nplanes = p;
        T->h = h;
        double sum = 0.0;
        double is2 = 1.0 / (2.0 * s.sigma[0] * s.sigma[0]);
        for (int v = -h; v <= h; ++v)
            for (int u = -h; u <= h; ++u) sum += exp(-(double)(u * u + v * v) * is2);
        S0 = sum;
    }
    __syncthreads();
    const int nb = T->nb;
    int k = threadIdx.x;
    if (k < nb) {
        double is2 = 1.0 / (2.0 * s.sigma[kg[k]] * s.sigma[kg[k]]);
        double is20 = 1.0 / (2.0 * s.sigma[0] * s.sigma[0]);
        double raw_sum = 0.0;
        for (int v = -h; v <= h; ++v)
            for (int u = -h; u <= h; ++u)
                raw_sum += exp(-(double)(u * u + v * v) * is2) * pow((double)u, ki[k]) *
                           pow((double)v, kj[k]);
        bool even = (ki[k] % 2 == 0) && (kj[k] % 2 == 0);
        double c0 = (k >= 1 && even) ? raw_sum / S0 : 0.0;   // subtract c0 * B_0raw
        double nrm = 0.0;
        for (int v = -h; v <= h; ++v)
            for (int u = -h; u <= h; ++u) {
                double b = exp(-(double)(u * u + v * v) * is2) * pow((double)u, ki[k]) *
                           pow((double)v, kj[k]) - c0 * exp(-(double)(u * u + v * v) * is20);
                nrm += b * b;
            }
        double a, be;
        if (k == 0) {
            a = 1.0 / S0;
            be = 0.0;
        } else {
            a = 1.0 / sqrt(nrm);
            be = -c0 * a;
        }
        alpha[k] = a;
        beta[k] = be;
        T->gam[k] = (float)(be * S0);     // C'_k = alpha_k conv_k + (beta_k / alpha_0) C'_0
        T->kpl[k] = kp[k];
        for (int v = -h; v <= h; ++v)
            T->colf[k][v + h] = (float)(a * exp(-(double)(v * v) * is2) * pow((double)v, kj[k]));
    }
    __syncthreads();
    // 2-D normalised basis for the kernel expansion
    for (int idx = threadIdx.x; idx < nb * K * K; idx += blockDim.x) {
        int kk = idx / (K * K), t = idx % (K * K);
        int v = t / K - h, u = t % K - h;
        double is2 = 1.0 / (2.0 * s.sigma[kg[kk]] * s.sigma[kg[kk]]);
        double is20 = 1.0 / (2.0 * s.sigma[0] * s.sigma[0]);
        double b = exp(-(double)(u * u + v * v) * is2) * pow((double)u, ki[kk]) * pow((double)v, kj[kk]);
        T->b2d[kk][t] = alpha[kk] * b + beta[kk] * exp(-(double)(u * u + v * v) * is20);
    }
    // row filters per plane (g, i)
    if (threadIdx.x < 32) {
        int p = threadIdx.x;
        int pp = 0;
        for (int g = 0; g < s.n_gauss; ++g)
            for (int i = 0; i <= s.degree[g]; ++i, ++pp)
                if (pp == p) {
                    T->ipow[p] = i;
                    double is2 = 1.0 / (2.0 * s.sigma[g] * s.sigma[g]);
                    for (int u = -h; u <= h; ++u)
                        T->rowf[p][u + h] = (float)(exp(-(double)(u * u) * is2) * pow((double)u, i));
                }
    }
}

// Sum consecutive groups of partial vectors in a fixed order (deterministic).
__global__ void sum_parts_kernel(const double *in, int stride, int n_in, int group, double *out) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int set = blockIdx.y;
    if (e >= stride) return;
    int j0 = set * group, j1 = min(j0 + group, n_in);
    double s = 0.0;
    for (int j = j0; j < j1; ++j) s += in[(size_t)j * stride + e];
    out[(size_t)set * stride + e] = s;
}

// ---------------------------------------------------------------------------
// Solve: assemble A and b from the moments, Jacobi scale, right-looking
// Cholesky on the packed lower triangle, two triangular solves.
struct SolveArgs {
    const double *sums;        // [n_solves][stride]
    int stride;
    int nb, D, Dbg, n;
    double *coeffs;
    int64_t *n_fit;
    int32_t *status;
    double *gtri;              // global fallback storage for the factor (or null)
};

__device__ __forceinline__ void unpack_row(int r, int nb, int D, int Dbg, int &k, int &p, int &q) {
    int nP = (D + 1) * (D + 2) / 2;
    int m;
    int Dm;
    if (r < nb * nP) { k = r / nP; m = r % nP; Dm = D; }
    else { k = nb; m = r - nb * nP; Dm = Dbg; }
    // monomial m of degree <= Dm: p outer, q inner
    int pp = 0;
    while (m > Dm - pp) { m -= Dm - pp + 1; ++pp; }
    p = pp;
    q = m;
}

__device__ __forceinline__ double gram_at(const double *G, int q, int k, int l) {
    // G[q][bp][16][16], blocks (0,0), (0,1), (1,1) of the symmetric 32x32 moment
    if (k > l) { int t = k; k = l; l = t; }
    const double *g = G + (size_t)q * 768;
    if (l < 16) return g[k * 16 + l];
    if (k < 16) return g[256 + k * 16 + (l - 16)];
    return g[512 + (k - 16) * 16 + (l - 16)];
}

__device__ double block_sum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    return s;
}

constexpr int SOLVE_THREADS = 1024;

// One workgroup of SOLVE_THREADS per solve.  Rows of the packed triangle are
// addressed through a table of row offsets; a wave walks a row with its
// lanes on consecutive columns (contiguous in the packed storage).  The
// factorisation takes one barrier per two columns: a phase applies the
// unscaled columns j and j + 1 to the trailing matrix in one pass and scales
// the previous phase's two columns, which no thread reads during the phase.
// GLT: the factor lives in global memory (a.gtri, for devices whose LDS is too
// small); otherwise it is in LDS and every access is a plain LDS instruction.
template <bool GLT>
__global__ __launch_bounds__(SOLVE_THREADS) void fit_solve_kernel(SolveArgs a) {
    constexpr int NT = SOLVE_THREADS, NWV = NT / 64;
    extern __shared__ double sl[];
    __shared__ int roff[256];             // r (r + 1) / 2 for r < n <= 192
    __shared__ short rk[256];             // basis, x-power and y-power of row r
    __shared__ unsigned char rp[256], rq[256];
    __shared__ double rdiag[256];         // 1 / L_ii
    __shared__ double tcol[2][256];       // column j + 1 after column j, by phase parity
    const int n = a.n, tid = threadIdx.x, sol = blockIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int ntri = n * (n + 1) / 2;
    double *L = GLT ? a.gtri + (size_t)sol * ntri : sl;
    double *bb = sl + (GLT ? 0 : ntri);
    double *dd = bb + n;
    double *red = dd + n;                 // [NWV]
    __shared__ int bad;
    const double *sums = a.sums + (size_t)sol * a.stride;
    const int D = a.D, NQ = (2 * D + 1) * (2 * D + 2) / 2;
    const double cnt = sums[(size_t)NQ * 768 + (D + 1) * (D + 2) / 2 * 32];
    double *co = a.coeffs + (size_t)sol * n;
    if (tid == 0) {
        bad = 0;
        if (a.n_fit) a.n_fit[sol] = (int64_t)cnt;
    }
    if (cnt < (double)n) {
        for (int i = tid; i < n; i += NT) co[i] = __builtin_nan("");
        if (tid == 0) a.status[sol] = ARGUS_ETOOFEW;
        return;
    }
    for (int r = tid; r < n; r += NT) {
        int k, p, q;
        unpack_row(r, a.nb, D, a.Dbg, k, p, q);
        roff[r] = r * (r + 1) / 2;
        rk[r] = (short)k;
        rp[r] = (unsigned char)p;
        rq[r] = (unsigned char)q;
    }
    __syncthreads();
    // assemble the packed lower triangle and the rhs
    for (int r = wv; r < n; r += NWV) {
        const int kr = rk[r], pr = rp[r], qr = rq[r];
        for (int c = lane; c <= r; c += 64)
            L[roff[r] + c] = gram_at(sums, qidx(pr + rp[c], qr + rq[c], 2 * D), kr, rk[c]);
    }
    for (int r = tid; r < n; r += NT) bb[r] = sums[(size_t)NQ * 768 + qidx(rp[r], rq[r], D) * 32 + rk[r]];
    __syncthreads();
    for (int r = tid; r < n; r += NT) {
        double dg = L[roff[r] + r];
        if (!(dg > 0.0)) bad = 1;
        dd[r] = dg > 0.0 ? 1.0 / sqrt(dg) : 0.0;
    }
    __syncthreads();
    if (bad) {
        for (int i = tid; i < n; i += NT) co[i] = __builtin_nan("");
        if (tid == 0) a.status[sol] = ARGUS_ESINGULAR;
        return;
    }
    // Jacobi scaling
    for (int r = wv; r < n; r += NWV) {
        const double dr = dd[r];
        for (int c = lane; c <= r; c += 64) L[roff[r] + c] *= dr * dd[c];
    }
    for (int r = tid; r < n; r += NT) bb[r] *= dd[r];
    __syncthreads();
    double mx = 0.0;
    for (int r = tid; r < n; r += NT) mx = fmax(mx, L[roff[r] + r]);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (lane == 0) red[wv] = mx;
    __syncthreads();
    double maxdiag = 0.0;
    for (int i = 0; i < NWV; ++i) maxdiag = fmax(maxdiag, red[i]);
    const double tol = (double)n * 0x1p-52 * maxdiag;
    __syncthreads();
    // Right-looking Cholesky, two columns per barrier.  A phase takes columns
    // j and j + 1 as they stand (updated by every earlier column) and applies
    // both to the trailing rows and columns c >= j + 2 in one pass:
    //   t_i = a_i,j+1 - a_ij a_j+1,j / a_jj          (column j + 1 after column j)
    //   p1  = a_j+1,j+1 - a_j+1,j^2 / a_jj           (its pivot)
    //   a_ic -= a_ij a_cj / a_jj + t_i t_c / p1      (c <= i)
    // Every thread forms p1 itself and t_c on the fly from the two columns,
    // which nobody writes during the phase (t_i goes to tcol), so the phase
    // needs no barrier inside.  tcol alternates between two buffers: a phase
    // writes one while the scaling at its start still reads the other.  The columns are scaled to L at the start of
    // the next phase: L_ij = a_ij / sqrt(a_jj), L_i,j+1 = t_i / sqrt(p1); the
    // diagonals stay as they are and the substitutions use rdiag = 1 / L_jj.
    double pv0 = 0.0, pv1 = 0.0;         // pivots of the previous phase
    for (int j = 0;; j += 2) {
        if (j > 0) {
            const int c0 = j - 2;
            const double rs0 = 1.0 / sqrt(pv0), rs1 = 1.0 / sqrt(pv1);
            for (int i = c0 + 1 + tid; i < n; i += NT) L[roff[i] + c0] *= rs0;
            const double *tp = tcol[((j >> 1) - 1) & 1];
            for (int i = c0 + 2 + tid; i < n; i += NT) L[roff[i] + c0 + 1] = tp[i] * rs1;
            if (tid == 0) {
                rdiag[c0] = rs0;
                rdiag[c0 + 1] = rs1;
            }
        }
        if (j >= n) break;
        const double piv = L[roff[j] + j];
        if (!(piv > tol)) {
            if (tid == 0) bad = 1;
            break;
        }
        if (j == n - 1) {                  // odd count: the last column alone
            if (tid == 0) rdiag[j] = 1.0 / sqrt(piv);
            break;
        }
        const double ip = 1.0 / piv;
        const double r = L[roff[j + 1] + j] * ip;
        const double p1 = L[roff[j + 1] + j + 1] - L[roff[j + 1] + j] * r;
        if (!(p1 > tol)) {
            if (tid == 0) bad = 1;
            break;
        }
        const double ip1 = 1.0 / p1;
        // rows i >= j + 2, a wave per row, its lanes on consecutive columns
        double *tw = tcol[(j >> 1) & 1];
        for (int i = j + 2 + wv; i < n; i += NWV) {
            double *Li = L + roff[i];
            const double lij = Li[j];
            const double ti = Li[j + 1] - lij * r;
            if (lane == 0) tw[i] = ti;
            const double a0 = lij * ip, a1 = ti * ip1;
            for (int c = j + 2 + lane; c <= i; c += 64) {
                const double lcj = L[roff[c] + j];
                const double tc = L[roff[c] + j + 1] - lcj * r;
                Li[c] -= a0 * lcj + a1 * tc;
            }
        }
        pv0 = piv;
        pv1 = p1;
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        for (int i = tid; i < n; i += NT) co[i] = __builtin_nan("");
        if (tid == 0) a.status[sol] = ARGUS_ESINGULAR;
        return;
    }
    // forward and back substitution (wave 0)
    if (tid < 64) {
        for (int i = 0; i < n; ++i) {
            double s = 0.0;
            for (int k = tid; k < i; k += 64) s += L[roff[i] + k] * bb[k];
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            double v = (bb[i] - s) * rdiag[i];
            __builtin_amdgcn_wave_barrier();
            bb[i] = v;      // every lane stores the same value, so each lane sees it
            __builtin_amdgcn_wave_barrier();
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1 + tid; k < n; k += 64) s += L[roff[k] + i] * bb[k];
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
            double v = (bb[i] - s) * rdiag[i];
            __builtin_amdgcn_wave_barrier();
            bb[i] = v;
            __builtin_amdgcn_wave_barrier();
        }
        for (int i = tid; i < n; i += 64) co[i] = dd[i] * bb[i];
        if (tid == 0) a.status[sol] = ARGUS_OK;
    }
}

// K_m = sum_k a_{k nP + m} B_k (FP64), bg_m = a_{nb nP + m}
__global__ void expand_kernel(const BasisTables *T, const double *coeffs, int n, int nP, int nPb,
                              float *stamps, float *bg) {
    const int s = blockIdx.x / nP, m = blockIdx.x % nP;
    const int K = 2 * T->h + 1, nb = T->nb;
    const double *a = coeffs + (size_t)s * n;
    for (int t = threadIdx.x; t < K * K; t += blockDim.x) {
        double acc = 0.0;
        for (int k = 0; k < nb; ++k) acc += a[k * nP + m] * T->b2d[k][t];
        stamps[((size_t)s * nP + m) * K * K + t] = (float)acc;
    }
    if (threadIdx.x == 0 && m < nPb) bg[(size_t)s * nPb + m] = (float)a[nb * nP + m];
}

template <int D>
int fit_launch_d(argus_ctx *ctx, argus_dims d, const argus_kernel_spec *spec, FitArgs &fa,
                 int n_regions, int parts_per_region, double **sums_out) {
    using S = FitShape<D>;
    fa.stride = S::NQ * 768 + S::NR * 32 + 1;
    fa.stride = (fa.stride + 1) & ~1;
    const int n_parts = n_regions * parts_per_region;
    const int group = 64;
    const int n_g1 = spec->mode == ARGUS_FIT_GLOBAL ? (n_parts + group - 1) / group : 0;
    const int n = fa.nb * argus_npoly(D) + argus_npoly(spec->bg_degree);
    size_t need = ((size_t)n_parts + n_g1 + n_regions) * fa.stride * sizeof(double) +
                  (size_t)n * (n + 1) / 2 * sizeof(double) * n_regions;
    int rc = argus_ws_reserve(ctx, need + 256);
    if (rc) return rc;
    double *base = (double *)ctx->ws;
    fa.partials = base;
    double *stage1 = base + (size_t)n_parts * fa.stride;
    double *sums = stage1 + (size_t)n_g1 * fa.stride;
    dim3 grid(fa.RX * fa.spt, fa.RY * fa.rchunks);
    argus_time_begin(ctx);
    switch (spec->precision) {
        case ARGUS_FP64: rc = fit_accum_launch_fp64(ctx, fa, D, grid); break;
        case ARGUS_BF16X3: rc = fit_accum_launch_bf16x3(ctx, fa, D, grid); break;
        default: rc = fit_accum_launch_fp32(ctx, fa, D, grid); break;
    }
    if (rc) return rc;
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "fit_accum");
    argus_time_begin(ctx);
    dim3 rb((fa.stride + 255) / 256);
    if (spec->mode == ARGUS_FIT_GLOBAL) {
        hipLaunchKernelGGL(sum_parts_kernel, dim3(rb.x, n_g1), dim3(256), 0, ctx->stream,
                           (const double *)fa.partials, fa.stride, n_parts, group, stage1);
        hipLaunchKernelGGL(sum_parts_kernel, dim3(rb.x, 1), dim3(256), 0, ctx->stream,
                           (const double *)stage1, fa.stride, n_g1, n_g1, sums);
    } else {
        hipLaunchKernelGGL(sum_parts_kernel, dim3(rb.x, n_regions), dim3(256), 0, ctx->stream,
                           (const double *)fa.partials, fa.stride, n_parts, parts_per_region, sums);
    }
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "fit_reduce");
    *sums_out = sums;
    return ARGUS_OK;
}

}  // namespace

int launch_basis_tables_to(argus_ctx *ctx, const argus_kernel_spec *spec, BasisTables *dst) {
    hipLaunchKernelGGL(basis_tables_kernel, dim3(1), dim3(256), 0, ctx->stream, *spec, dst);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

int launch_basis_tables(argus_ctx *ctx, const argus_kernel_spec *spec) {
    const argus_kernel_spec &o = ctx->tables_spec;
    bool same = ctx->tables_valid && o.n_gauss == spec->n_gauss && o.half_width == spec->half_width;
    for (int g = 0; same && g < spec->n_gauss; ++g)
        same = o.sigma[g] == spec->sigma[g] && o.degree[g] == spec->degree[g];
    if (same) return ARGUS_OK;
    hipLaunchKernelGGL(basis_tables_kernel, dim3(1), dim3(256), 0, ctx->stream, *spec, ctx->tables);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    ctx->tables_spec = *spec;
    ctx->tables_valid = true;
    return ARGUS_OK;
}

int launch_fit(argus_ctx *ctx, argus_dims d, const argus_kernel_spec *spec, const float *ref,
               const float *ref_var, const uint8_t *ref_mask, const float *sci,
               const float *sci_var, const uint8_t *sci_mask, double *coeffs, int64_t *n_fit,
               int32_t *status) {
    FitArgs fa;
    fa.ref = ref; fa.rvar = ref_var; fa.sci = sci; fa.svar = sci_var;
    fa.rmask = ref_mask; fa.smask = sci_mask;
    fa.tab = ctx->tables;
    fa.pitch = d.pitch; fa.W = d.width; fa.H = d.height;
    fa.h = spec->half_width;
    fa.nb = argus_nbasis(spec);
    fa.nplanes = argus_nplanes(spec);
    // planes to the convolution waves, longest first onto the least loaded
    // wave: 8 waves (wave 0 at most 1 plane, the others at most 2) or 4 waves
    // (at most 4 each); at most 13 planes fit the basis limit.  Cost of a plane in VALU operations per pixel
    // row with paired symmetric taps: its row filter (h + 1), the paired
    // window of its column (2h, or h when it feeds one even filter) and h + 2
    // per column filter it feeds; wave 0 also stages the fit-set weights.
    {
        const int h = spec->half_width;
        int cost[ARGUS_MAX_PLANES];
        int p = 0;
        for (int g = 0; g < spec->n_gauss; ++g)
            for (int i = 0; i <= spec->degree[g]; ++i, ++p) {
                const int nk = spec->degree[g] - i + 1;
                cost[p] = (h + 1) + (nk > 1 ? 2 * h : h) + nk * (h + 2);
            }
        // 4 convolution waves (FP64 form), up to 4 planes each
        int load[4] = {3 * h, 0, 0, 0}, nin[4] = {};
        bool used[ARGUS_MAX_PLANES] = {};
        for (int w = 0; w < 4; ++w)
            for (int j = 0; j < 4; ++j) fa.plist[w][j] = -1;
        for (int n = 0; n < fa.nplanes; ++n) {
            int best = -1;
            for (int q = 0; q < fa.nplanes; ++q)
                if (!used[q] && (best < 0 || cost[q] > cost[best])) best = q;
            int w = -1;
            for (int c = 0; c < 4; ++c)
                if (nin[c] < 4 && (w < 0 || load[c] < load[w])) w = c;
            used[best] = true;
            fa.plist[w][nin[w]++] = (int8_t)best;
            load[w] += cost[best];
        }
        // 8 convolution waves (FP32 and BF16x3 forms)
        int load8[8] = {}, nin8[8] = {};
        load8[0] = 3 * h;
        bool used8[ARGUS_MAX_PLANES] = {};
        for (int w = 0; w < 8; ++w)
            for (int j = 0; j < 2; ++j) fa.plist8[w][j] = -1;
        for (int n = 0; n < fa.nplanes; ++n) {
            int best = -1;
            for (int q = 0; q < fa.nplanes; ++q)
                if (!used8[q] && (best < 0 || cost[q] > cost[best])) best = q;
            int w = -1;
            for (int c = 0; c < 8; ++c)
                if (nin8[c] < (c == 0 ? 1 : 2) && (w < 0 || load8[c] < load8[w])) w = c;
            used8[best] = true;
            fa.plist8[w][nin8[w]++] = (int8_t)best;
            load8[w] += cost[best];
        }
    }
    const bool global = spec->mode == ARGUS_FIT_GLOBAL;
    fa.RX = global ? 1 : spec->tiles_x;
    fa.RY = global ? 1 : spec->tiles_y;
    int maxw = (d.width + fa.RX - 1) / fa.RX;
    int maxh = (d.height + fa.RY - 1) / fa.RY;
    fa.spt = (maxw + SW - 1) / SW;
    // Row chunks: one workgroup runs per CU at a time, so the accumulation
    // takes ceil(workgroups / CUs) rounds of (rows per chunk + 2h halo rows)
    // steps each.  Take the chunk count (chunks no shorter than 8h) with the
    // shortest such makespan, which also avoids a last round that leaves
    // most CUs idle.
    {
        const int base = fa.RX * fa.RY * fa.spt;
        const int maxc = maxh / (8 * fa.h) > 1 ? maxh / (8 * fa.h) : 1;
        const int ncu = ctx->n_cu > 0 ? ctx->n_cu : 256;
        int64_t best = -1;
        fa.rchunks = 1;
        for (int c = 1; c <= maxc; ++c) {
            const int64_t rounds = ((int64_t)base * c + ncu - 1) / ncu;
            const int64_t t = rounds * ((maxh + c - 1) / c + 2 * fa.h);
            if (best < 0 || t < best) {
                best = t;
                fa.rchunks = c;
            }
        }
    }
    fa.sx = d.width > 1 ? 2.0 / (d.width - 1) : 0.0;
    fa.sy = d.height > 1 ? 2.0 / (d.height - 1) : 0.0;
    const int n_regions = fa.RX * fa.RY;
    const int parts_per_region = fa.rchunks * fa.spt;
    double *sums = nullptr;
    int rc;
    switch (spec->spatial_degree) {
        case 0: rc = fit_launch_d<0>(ctx, d, spec, fa, n_regions, parts_per_region, &sums); break;
        case 1: rc = fit_launch_d<1>(ctx, d, spec, fa, n_regions, parts_per_region, &sums); break;
        default: rc = fit_launch_d<2>(ctx, d, spec, fa, n_regions, parts_per_region, &sums); break;
    }
    if (rc) return rc;
    SolveArgs sa;
    sa.sums = sums;
    sa.stride = fa.stride;
    sa.nb = fa.nb;
    sa.D = spec->spatial_degree;
    sa.Dbg = spec->bg_degree;
    sa.n = fa.nb * argus_npoly(sa.D) + argus_npoly(sa.Dbg);
    sa.coeffs = coeffs;
    sa.n_fit = n_fit;
    sa.status = status;
    sa.gtri = nullptr;
    size_t lds = ((size_t)sa.n * (sa.n + 1) / 2 + 2 * sa.n + SOLVE_THREADS / 64) * sizeof(double);
    int dev_max = 0;
    ARGUS_HIP_CHECK(ctx, hipDeviceGetAttribute(&dev_max, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                               ctx->device));
    hipFuncAttributes fattr;
    ARGUS_HIP_CHECK(ctx, hipFuncGetAttributes(&fattr, (const void *)fit_solve_kernel<false>));
    if (lds + fattr.sharedSizeBytes > (size_t)dev_max) {
        // factor in global memory (after the sums in the workspace)
        size_t tri = (size_t)sa.n * (sa.n + 1) / 2 * sizeof(double) * n_regions;
        size_t used = (size_t)((char *)(sums + (size_t)n_regions * fa.stride) - (char *)ctx->ws);
        if (used + tri > ctx->ws_bytes)
            return argus_fail(ctx, ARGUS_ENOMEM, "solve storage does not fit the workspace");
        sa.gtri = sums + (size_t)n_regions * fa.stride;
        lds = ((size_t)2 * sa.n + SOLVE_THREADS / 64) * sizeof(double);
    }
    const void *kfn = sa.gtri ? (const void *)fit_solve_kernel<true> : (const void *)fit_solve_kernel<false>;
    ARGUS_HIP_CHECK(ctx, hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    argus_time_begin(ctx);
    if (sa.gtri)
        hipLaunchKernelGGL(fit_solve_kernel<true>, dim3(n_regions), dim3(SOLVE_THREADS), lds, ctx->stream, sa);
    else
        hipLaunchKernelGGL(fit_solve_kernel<false>, dim3(n_regions), dim3(SOLVE_THREADS), lds, ctx->stream, sa);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "fit_solve");
    return ARGUS_OK;
}

namespace {
__global__ void chi2_failed_kernel(double *chi2, const int32_t *status, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && status[i] != ARGUS_OK) chi2[i] = __builtin_nan("");
}
}  // namespace

int launch_chi2_failed(argus_ctx *ctx, double *chi2, const int32_t *status, int n) {
    hipLaunchKernelGGL(chi2_failed_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, chi2,
                       status, n);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}

int launch_expand(argus_ctx *ctx, const argus_kernel_spec *spec, const double *coeffs,
                  float *stamps, float *bg) {
    int n, ns;
    argus_kernel_dims(spec, &n, &ns);
    int nP = argus_npoly(spec->spatial_degree), nPb = argus_npoly(spec->bg_degree);
    hipLaunchKernelGGL(expand_kernel, dim3(ns * nP), dim3(256), 0, ctx->stream,
                       (const BasisTables *)ctx->tables, coeffs, n, nP, nPb, stamps, bg);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    return ARGUS_OK;
}
