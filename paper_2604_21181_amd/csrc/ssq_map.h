// Sauter-Schwab maps for coincident, common-edge and common-vertex pairs
// of triangles (Sec. 4.2 and 6.1), shared by the fill and its adjoint.
#pragma once

#include "p2_device.h"

namespace mbem {

// Maps of [0,1]^4 -> Th x Th, Th = {0 <= t <= s <= 1}; the common edge is
// {t = 0} with the same s in both triangles, the common vertex is (0,0).
// Returns the Jacobian of the region's map.
__device__ inline double ss_region(int cls, int r, double u, double e1, double e2,
                                   double e3, double &s1, double &t1, double &s2,
                                   double &t2) {
    const double u3 = u * u * u;
    if (cls == 3) {
        const double a = e1 * e2, b = a * e3;
        switch (r) {
        case 0: s1 = u; t1 = u * (1 - e1 + a); s2 = u * (1 - b); t2 = u * (1 - e1); break;
        case 1: s1 = u * (1 - b); t1 = u * (1 - e1); s2 = u; t2 = u * (1 - e1 + a); break;
        case 2: s1 = u; t1 = u * e1 * (1 - e2 + e2 * e3); s2 = u * (1 - a); t2 = u * e1 * (1 - e2); break;
        case 3: s1 = u * (1 - a); t1 = u * e1 * (1 - e2); s2 = u; t2 = u * e1 * (1 - e2 + e2 * e3); break;
        case 4: s1 = u * (1 - b); t1 = u * e1 * (1 - e2 * e3); s2 = u; t2 = u * e1 * (1 - e2); break;
        default: s1 = u; t1 = u * e1 * (1 - e2); s2 = u * (1 - b); t2 = u * e1 * (1 - e2 * e3); break;
        }
        return u3 * e1 * e1 * e2;
    }
    if (cls == 2) {
        const double a = e1 * e2, b = a * e3;
        switch (r) {
        case 0: s1 = u; t1 = u * e1 * e3; s2 = u * (1 - a); t2 = u * e1 * (1 - e2); return u3 * e1 * e1;
        case 1: s1 = u; t1 = u * e1; s2 = u * (1 - b); t2 = u * a * (1 - e3); break;
        case 2: s1 = u * (1 - a); t1 = u * e1 * (1 - e2); s2 = u; t2 = u * b; break;
        case 3: s1 = u * (1 - b); t1 = u * a * (1 - e3); s2 = u; t2 = u * e1; break;
        default: s1 = u * (1 - b); t1 = u * e1 * (1 - e2 * e3); s2 = u; t2 = u * a; break;
        }
        return u3 * e1 * e1 * e2;
    }
    if (r == 0) { s1 = u; t1 = u * e1; s2 = u * e2; t2 = u * e2 * e3; }
    else        { s1 = u * e2; t1 = u * e2 * e3; s2 = u; t2 = u * e1; }
    return u3 * e2;
}

// (s,t) of Th in the re-indexed triangle -> (xi, eta) of the stored one.
// code holds the stored local vertex of re-indexed vertex k in bits 2k.
__device__ inline void ss_local(int code, double s, double t, double &xi, double &eta) {
    const double L[3] = {1.0 - s, s - t, t};
    double l[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) l[(code >> (2 * k)) & 3] = L[k];
    xi = l[1];
    eta = l[2];
}

}  // namespace mbem
