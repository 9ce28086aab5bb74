// Host-side mapping helpers: halo-extended cell centres of the paper's grid
// families, with the ghost rows beyond each wall holding the symmetrically
// continued geometry (Sec. 3.1): each ghost row is the mirror image of an
// interior row across the wall, repeated when the halo is wider than the
// channel.  Planar channels take wall-normal faces (uniform, App. C
// contraction, geometric stretching); polar annuli use the half-spaced
// (r, theta) lattice of App. D.  No device code; errors are returned as text.
#pragma once

#include <cmath>
#include <cstdint>
#include <new>
#include <string>

namespace lbm_maps {

// Position of 1-based row k on the reflected wall-normal line: centres
// c[0..n1-1] between the walls lo and hi.
inline double reflected(const double *c, int n1, double lo, double hi, long k)
{
    if (k < 1) return 2.0 * lo - reflected(c, n1, lo, hi, 1 - k);
    if (k > n1) return 2.0 * hi - reflected(c, n1, lo, hi, 2L * n1 + 1 - k);
    return c[k - 1];
}

// Fills the n1 + 2 halo reflected centres of the faces f[0..n1] into line[]
// (row r holds 1-based row r - halo + 1).  Returns an empty string or the error.
inline std::string wall_normal_line(int32_t n1, int32_t halo, const double *f, double *line)
{
    for (int k = 0; k <= n1; ++k)
        if (!std::isfinite(f[k])) return "faces must be finite";
    for (int k = 0; k < n1; ++k)
        if (!(f[k + 1] > f[k])) return "faces must increase strictly";
    double *c = new (std::nothrow) double[n1];
    if (!c) return "out of host memory";
    for (int k = 0; k < n1; ++k) c[k] = 0.5 * (f[k + 1] + f[k]);
    for (long r = 0; r < (long)n1 + 2L * halo; ++r)
        line[r] = reflected(c, n1, f[0], f[n1], r - halo + 1);
    delete[] c;
    return std::string();
}

inline std::string check_shape(int32_t n1, int32_t n2, int32_t halo, const void *f, const void *x, const void *y)
{
    if (!f || !x || !y) return "null pointer";
    if (n1 < 1 || n2 < 1) return "n1 and n2 must be at least 1";
    if (halo < 1 || halo > 64) return "halo must be 1..64";
    if ((double)(n1 + 2.0 * halo) * (n2 + 2.0 * halo) > (double)(1LL << 31)) return "grid too large";
    return std::string();
}

// Planar channel: wall-normal coordinate x from the faces, periodic
// coordinate y = (j + 1/2) d_per, j = -halo .. n2 + halo - 1.
inline std::string map_planar(int32_t n1, int32_t n2, int32_t halo, const double *faces, double d_per, double *x,
                              double *y)
{
    std::string e = check_shape(n1, n2, halo, faces, x, y);
    if (!e.empty()) return e;
    if (!(d_per > 0.0) || !std::isfinite(d_per)) return "periodic spacing must be finite and > 0";
    const long R = n1 + 2L * halo, C = n2 + 2L * halo;
    double *line = new (std::nothrow) double[R];
    if (!line) return "out of host memory";
    e = wall_normal_line(n1, halo, faces, line);
    if (e.empty())
        for (long r = 0; r < R; ++r)
            for (long j = 0; j < C; ++j) {
                x[r * C + j] = line[r];
                y[r * C + j] = ((double)(j - halo) + 0.5) * d_per;
            }
    delete[] line;
    return e;
}

// Polar annulus: radius from the radial faces (every ring, ghosts included,
// must have r > 0), angle theta_j = (j + 1/2) 2 pi / ntheta; n2 <= ntheta
// columns are kept and continued with the true angular step.
inline std::string map_polar(int32_t n1, int32_t n2, int32_t halo, const double *r_faces, int32_t ntheta, double *x,
                             double *y)
{
    std::string e = check_shape(n1, n2, halo, r_faces, x, y);
    if (!e.empty()) return e;
    if (ntheta < 1 || n2 > ntheta) return "need 1 <= n2 <= ntheta";
    const long R = n1 + 2L * halo, C = n2 + 2L * halo;
    double *line = new (std::nothrow) double[R];
    if (!line) return "out of host memory";
    e = wall_normal_line(n1, halo, r_faces, line);
    if (e.empty())
        for (long r = 0; r < R; ++r)
            if (!(line[r] > 0.0)) {
                e = "inner radius too small for the ghost layers";
                break;
            }
    if (e.empty()) {
        const double dth = 2.0 * M_PI / ntheta;
        for (long r = 0; r < R; ++r)
            for (long j = 0; j < C; ++j) {
                const double th = ((double)(j - halo) + 0.5) * dth;
                x[r * C + j] = line[r] * std::cos(th);
                y[r * C + j] = line[r] * std::sin(th);
            }
    }
    delete[] line;
    return e;
}

} // namespace lbm_maps
