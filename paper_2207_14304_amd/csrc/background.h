// Bilinear evaluation of the median-filtered background grid at a pixel
// (shared by the background map and the source detection).
//
// Cells are box x box from the origin; the last cell of an axis spans the
// remainder.  Nodes sit at cell centres, (x0 + x1 - 1)/2 for a cell spanning
// [x0, x1); between two nodes the value is interpolated linearly per axis
// (a + t (b - a), exact on a constant grid); before the first and after the
// last node it is held constant.
#pragma once
#include <hip/hip_runtime.h>

struct BgGrid {
    const float *grid;         // [gy][gx]
    int box, gx, gy;
    float cxl, cyl;            // centre of the last cell column / row
};

inline BgGrid make_bg_grid(const float *grid, int box, int W, int H) {
    BgGrid g;
    g.grid = grid;
    g.box = box;
    g.gx = (W + box - 1) / box;
    g.gy = (H + box - 1) / box;
    g.cxl = 0.5f * (float)((g.gx - 1) * box + W - 1);
    g.cyl = 0.5f * (float)((g.gy - 1) * box + H - 1);
    return g;
}

// left node and weight of the right node along one axis
__device__ __forceinline__ void bg_axis(int x, int box, int n, float clast, int &i, float &t) {
    const float c0 = 0.5f * (float)(box - 1);
    const float xf = (float)x;
    if (xf < c0 || n == 1) { i = 0; t = 0.f; return; }
    if (xf >= clast) { i = n - 1; t = 0.f; return; }
    i = (int)((xf - c0) / (float)box);      // non-negative: truncation is the floor
    if (i > n - 2) i = n - 2;
    const float ci = (float)(i * box) + c0;
    const float cn = (i + 1 == n - 1) ? clast : ci + (float)box;
    t = (xf - ci) / (cn - ci);
}

__device__ __forceinline__ float bg_at(const BgGrid &g, int x, int y) {
    int ix, iy;
    float tx, ty;
    bg_axis(x, g.box, g.gx, g.cxl, ix, tx);
    bg_axis(y, g.box, g.gy, g.cyl, iy, ty);
    const int ix1 = ix + 1 < g.gx ? ix + 1 : ix, iy1 = iy + 1 < g.gy ? iy + 1 : iy;
    const float *r0 = g.grid + (size_t)iy * g.gx, *r1 = g.grid + (size_t)iy1 * g.gx;
    const float g00 = r0[ix], g01 = r0[ix1], g10 = r1[ix], g11 = r1[ix1];
    const float top = g00 + tx * (g01 - g00);
    const float bot = g10 + tx * (g11 - g10);
    return top + ty * (bot - top);
}
