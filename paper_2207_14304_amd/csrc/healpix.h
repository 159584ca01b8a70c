// HEALPix geometry and the gnomonic frame projection, for the host (tile
// enumeration) and the device (segment resampling).  FP64 throughout.
//
// The HEALPix projection maps the sphere to a plane (x_s, y_s) in which the
// twelve equal-area base pixels are diamonds of half-diagonal pi/4
// (Gorski et al. 2005; Calabretta & Roukema 2007):
//   |z| <= 2/3: x_s = phi, y_s = 3 pi z / 8;
//   |z| >  2/3: sigma = sqrt(3 (1 - |z|)), x_s = phi_c + (phi - phi_c) sigma,
//               y_s = sign(z) (pi/4) (2 - sigma), phi_c the centre of phi's
//               quadrant (pi/4 + k pi/2).
// Diamond centres: (pi/4 + f pi/2, pi/4) for f = 0..3, ((f-4) pi/2, 0) for
// f = 4..7, (pi/4 + (f-8) pi/2, -pi/4) for f = 8..11.  Face coordinates
// (a, b) in [0, 1]^2: x_s = x_c + (pi/4)(a - b), y_s = y_c + (pi/4)(a + b - 1).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "argus.h"

namespace argus_hp {

constexpr double PI = 3.14159265358979323846;
constexpr double QP = PI / 4, HP = PI / 2, TWO_PI = 2 * PI;

__host__ __device__ inline void face_centre(int f, double &xc, double &yc) {
    if (f < 4) { xc = QP + f * HP; yc = QP; }
    else if (f < 8) { xc = (f - 4) * HP; yc = 0.0; }
    else { xc = QP + (f - 8) * HP; yc = -QP; }
}

// plane point -> (z, phi), phi in [0, 2 pi)
__host__ __device__ inline void plane_to_sphere(double xs, double ys, double &z, double &phi) {
    xs = fmod(xs, TWO_PI);
    if (xs < 0) xs += TWO_PI;
    if (fabs(ys) <= QP) {
        z = ys * (8.0 / (3.0 * PI));
        phi = xs;
        return;
    }
    const double sig = 2.0 - fabs(ys) / QP;
    z = (ys > 0 ? 1.0 : -1.0) * (1.0 - sig * sig / 3.0);
    const double phic = QP + floor(xs / HP) * HP;
    phi = sig > 0 ? phic + (xs - phic) / sig : phic;
    phi = fmod(phi, TWO_PI);
    if (phi < 0) phi += TWO_PI;
}

// (z, phi) -> plane point
__host__ __device__ inline void sphere_to_plane(double z, double phi, double &xs, double &ys) {
    phi = fmod(phi, TWO_PI);
    if (phi < 0) phi += TWO_PI;
    if (fabs(z) <= 2.0 / 3.0) {
        xs = phi;
        ys = 3.0 * PI / 8.0 * z;
        return;
    }
    const double sig = sqrt(3.0 * (1.0 - fabs(z)));
    const double phic = QP + floor(phi / HP) * HP;
    xs = phic + (phi - phic) * sig;
    ys = (z > 0 ? 1.0 : -1.0) * QP * (2.0 - sig);
}

// plane point -> (face, a, b); face -1 if none (cannot happen on the image)
__host__ __device__ inline int plane_to_face(double xs, double ys, double &a, double &b) {
    xs = fmod(xs, TWO_PI);
    if (xs < 0) xs += TWO_PI;
    for (int f = 0; f < 12; ++f) {
        double xc, yc;
        face_centre(f, xc, yc);
        double dx = fmod(xs - xc + PI, TWO_PI);
        if (dx < 0) dx += TWO_PI;
        dx -= PI;
        const double u = dx / QP, v = (ys - yc) / QP;
        const double aa = 0.5 * (1 + u + v), bb = 0.5 * (1 - u + v);
        if (aa >= 0 && aa < 1 && bb >= 0 && bb < 1) {
            a = aa;
            b = bb;
            return f;
        }
    }
    return -1;
}

struct Wcs {
    double ra0, dec0;                 // radians
    double sd0, cd0;                  // sin, cos of dec0
    double crpix1, crpix2;
    double cd[4], cdi[4];             // degrees per pixel and its inverse
};

inline bool make_wcs(const argus_wcs &w, Wcs &o) {
    const double det = w.cd[0] * w.cd[3] - w.cd[1] * w.cd[2];
    if (!(det != 0.0) || !isfinite(det)) return false;
    o.ra0 = w.ra0 * PI / 180.0;
    o.dec0 = w.dec0 * PI / 180.0;
    o.sd0 = sin(o.dec0);
    o.cd0 = cos(o.dec0);
    o.crpix1 = w.crpix1;
    o.crpix2 = w.crpix2;
    for (int i = 0; i < 4; ++i) o.cd[i] = w.cd[i];
    o.cdi[0] = w.cd[3] / det;
    o.cdi[1] = -w.cd[1] / det;
    o.cdi[2] = -w.cd[2] / det;
    o.cdi[3] = w.cd[0] / det;
    return true;
}

// direction (z = sin dec, ra radians) -> frame pixel; returns the projection
// denominator (<= 0: the far side of the tangent plane)
__host__ __device__ inline double sky_to_pixel(const Wcs &w, double z, double ra, double &x,
                                               double &y) {
    const double cdd = sqrt(fmax(1.0 - z * z, 0.0));
    double s, c;
    sincos(ra - w.ra0, &s, &c);
    const double den = z * w.sd0 + cdd * w.cd0 * c;
    const double r2d = 180.0 / PI;
    const double xi = r2d * cdd * s / den;
    const double eta = r2d * (z * w.cd0 - cdd * w.sd0 * c) / den;
    x = w.cdi[0] * xi + w.cdi[1] * eta + w.crpix1;
    y = w.cdi[2] * xi + w.cdi[3] * eta + w.crpix2;
    return den;
}

// frame pixel -> direction (z = sin dec, ra radians in [0, 2 pi))
inline void pixel_to_sky(const Wcs &w, double x, double y, double &z, double &ra) {
    const double dx = x - w.crpix1, dy = y - w.crpix2;
    const double d2r = PI / 180.0;
    const double xi = d2r * (w.cd[0] * dx + w.cd[1] * dy);
    const double eta = d2r * (w.cd[2] * dx + w.cd[3] * dy);
    const double rho = hypot(xi, eta);
    const double cc = atan(rho);
    const double sc = sin(cc), ccs = cos(cc);
    const double sgn = rho > 0 ? eta * sc / rho : 0.0;
    z = ccs * w.sd0 + sgn * w.cd0;
    ra = w.ra0 + atan2(xi * sc, rho * w.cd0 * ccs - eta * w.sd0 * sc);
    ra = fmod(ra, TWO_PI);
    if (ra < 0) ra += TWO_PI;
}

}  // namespace argus_hp
