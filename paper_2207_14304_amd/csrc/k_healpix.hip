// Resampling of a calibrated frame into HEALPix-aligned segment images.
//
// A segment is one tile (face f, I, J) of NSIDE n; its m x m pixels are the
// HEALPix pixels of NSIDE n m inside the tile: pixel (p, q) (row q, column p)
// sits at face coordinates a = (I m + p + 1/2)/(n m), b = (J m + q + 1/2)/(n m).
// Per segment pixel (one thread, FP64 geometry): face coordinates -> HEALPix
// plane -> sphere -> gnomonic frame position -> bilinear interpolation of the
// frame (value: sum w cal; variance: sum w^2 var); NODATA where the position
// is off the frame (or behind the tangent plane) or any of the four
// neighbours is masked.  Consecutive threads take consecutive pixels of a
// segment row, so the stores are coalesced and the gathers of a wave fall on
// a few frame rows.
#include <algorithm>
#include <set>
#include <tuple>

#include "internal.h"
#include "healpix.h"

namespace {

using namespace argus_hp;

struct HpArgs {
    const float *cal, *var;
    const uint8_t *mask;
    const int32_t *tiles;              // [n][3]: face, I, J
    float *out, *outv;
    uint8_t *outm;
    Wcs w;
    int64_t pitch;
    int W, H, nside, m;
};

__global__ __launch_bounds__(256) void healpix_resample_kernel(HpArgs a) {
    const int p = blockIdx.x * 64 + (threadIdx.x & 63);
    const int q = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int t = blockIdx.z;
    if (p >= a.m || q >= a.m) return;
    const int f = a.tiles[3 * t], I = a.tiles[3 * t + 1], J = a.tiles[3 * t + 2];
    const double nm = (double)a.nside * a.m;
    const double fa = ((double)I * a.m + p + 0.5) / nm;
    const double fb = ((double)J * a.m + q + 0.5) / nm;
    double xc, yc;
    face_centre(f, xc, yc);
    double z, phi;
    plane_to_sphere(xc + QP * (fa - fb), yc + QP * (fa + fb - 1.0), z, phi);
    double x, y;
    const double den = sky_to_pixel(a.w, z, phi, x, y);
    float val = 0.f, vv = 0.f;
    uint8_t msk = ARGUS_NODATA;
    if (den > 0.0 && x >= 0.0 && x <= a.W - 1.0 && y >= 0.0 && y <= a.H - 1.0) {
        const int x0 = min((int)floor(x), max(a.W - 2, 0)), y0 = min((int)floor(y), max(a.H - 2, 0));
        const int x1 = min(x0 + 1, a.W - 1), y1 = min(y0 + 1, a.H - 1);
        const double fx = x - x0, fy = y - y0;
        const int64_t o00 = (int64_t)y0 * a.pitch + x0, o01 = (int64_t)y0 * a.pitch + x1;
        const int64_t o10 = (int64_t)y1 * a.pitch + x0, o11 = (int64_t)y1 * a.pitch + x1;
        const uint8_t m4 = a.mask[o00] | a.mask[o01] | a.mask[o10] | a.mask[o11];
        if (m4 == 0) {
            const double w00 = (1 - fx) * (1 - fy), w01 = fx * (1 - fy), w10 = (1 - fx) * fy,
                         w11 = fx * fy;
            val = (float)(w00 * a.cal[o00] + w01 * a.cal[o01] + w10 * a.cal[o10] + w11 * a.cal[o11]);
            vv = (float)(w00 * w00 * a.var[o00] + w01 * w01 * a.var[o01] +
                         w10 * w10 * a.var[o10] + w11 * w11 * a.var[o11]);
            msk = 0;
        }
    }
    const int64_t o = ((int64_t)t * a.m + q) * a.m + p;
    a.out[o] = val;
    a.outv[o] = vv;
    a.outm[o] = msk;
}

}  // namespace

int launch_resample_healpix(argus_ctx *ctx, argus_dims d, const float *cal, const float *var,
                            const uint8_t *mask, const argus_wcs *wcs, int nside, int m,
                            const int32_t *tiles, int n_tiles, float *out, float *out_var,
                            uint8_t *out_mask) {
    HpArgs a;
    if (!make_wcs(*wcs, a.w)) return argus_fail(ctx, ARGUS_EINVAL, "singular or non-finite cd matrix");
    a.cal = cal; a.var = var; a.mask = mask; a.tiles = tiles;
    a.out = out; a.outv = out_var; a.outm = out_mask;
    a.pitch = d.pitch; a.W = d.width; a.H = d.height; a.nside = nside; a.m = m;
    argus_time_begin(ctx);
    hipLaunchKernelGGL(healpix_resample_kernel, dim3((m + 63) / 64, (m + 3) / 4, n_tiles),
                       dim3(256), 0, ctx->stream, a);
    ARGUS_HIP_CHECK(ctx, hipGetLastError());
    argus_time_end(ctx, "healpix_resample");
    return ARGUS_OK;
}

// Tiles that the frame's pixels fall in, sampled every `step` pixels along
// both axes and along the last row and column.
int healpix_tiles(const argus_wcs *wcs, int W, int H, int nside, int step, int32_t *tiles,
                  int capacity, int *n_tiles) {
    Wcs w;
    if (!make_wcs(*wcs, w)) return ARGUS_EINVAL;
    std::set<std::tuple<int, int, int>> s;
    auto add = [&](int x, int y) {
        double z, ra, xs, ys, fa, fb;
        pixel_to_sky(w, x, y, z, ra);
        sphere_to_plane(z, ra, xs, ys);
        const int f = plane_to_face(xs, ys, fa, fb);
        if (f < 0) return;
        const int I = std::min((int)(fa * nside), nside - 1);
        const int J = std::min((int)(fb * nside), nside - 1);
        s.insert(std::make_tuple(f, I, J));
    };
    for (int y = 0;; y += step) {
        const int yy = std::min(y, H - 1);
        for (int x = 0;; x += step) {
            add(std::min(x, W - 1), yy);
            if (x >= W - 1) break;
        }
        if (y >= H - 1) break;
    }
    *n_tiles = (int)s.size();
    int i = 0;
    for (const auto &t : s) {
        if (i >= capacity) break;
        tiles[3 * i] = std::get<0>(t);
        tiles[3 * i + 1] = std::get<1>(t);
        tiles[3 * i + 2] = std::get<2>(t);
        ++i;
    }
    return ARGUS_OK;
}
