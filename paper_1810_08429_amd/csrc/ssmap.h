// The Sauter-Schwab regularising maps of [0,1]^4 onto T x T for touching
// triangle pairs, in full four-dimensional form (the single-layer product
// kernels use a dimension-reduced form of their own, quad.hip): the
// identical case in 6 regions, the common edge in 5, the common vertex in 2.
// (xi, e1, e2, e3) map to reference points (x1, x2) of the first and (y1, y2)
// of the second triangle, both parametrised as chi(s) = P0 + s1 (P1 - P0) +
// s2 (P2 - P1) with the shared vertex P0 = Q0 (and the shared edge P0 P1 =
// Q0 Q1); the return value is the Jacobian, which vanishes on the singular
// set to the order that cancels a kernel of order 1/r (single layer) or 1/r^2
// (double layer).
#pragma once

#include <hip/hip_runtime.h>

namespace gca {

enum { SS_IDENT = 0, SS_EDGE = 1, SS_VERT = 2 };

__device__ __forceinline__ int ss_nregions(int kase) { return kase == SS_IDENT ? 6 : (kase == SS_EDGE ? 5 : 2); }

__device__ inline double ss_map_full(int kase, int reg, double xi, double e1, double e2, double e3, double &x1,
                                     double &x2, double &y1, double &y2)
{
    if (kase == SS_IDENT) {
        switch (reg) {
        case 0: x1 = xi; x2 = xi * (1 - e1 + e1 * e2); y1 = xi * (1 - e1 * e2 * e3); y2 = xi * (1 - e1); break;
        case 1: x1 = xi * (1 - e1 * e2 * e3); x2 = xi * (1 - e1); y1 = xi; y2 = xi * (1 - e1 + e1 * e2); break;
        case 2: x1 = xi; x2 = xi * e1 * (1 - e2 + e2 * e3); y1 = xi * (1 - e1 * e2); y2 = xi * e1 * (1 - e2); break;
        case 3: x1 = xi * (1 - e1 * e2); x2 = xi * e1 * (1 - e2); y1 = xi; y2 = xi * e1 * (1 - e2 + e2 * e3); break;
        case 4: x1 = xi * (1 - e1 * e2 * e3); x2 = xi * e1 * (1 - e2 * e3); y1 = xi; y2 = xi * e1 * (1 - e2); break;
        default: x1 = xi; x2 = xi * e1 * (1 - e2); y1 = xi * (1 - e1 * e2 * e3); y2 = xi * e1 * (1 - e2 * e3); break;
        }
        return xi * xi * xi * e1 * e1 * e2;
    }
    if (kase == SS_EDGE) {
        switch (reg) {
        case 0:
            x1 = xi; x2 = xi * e1 * e3; y1 = xi * (1 - e1 * e2); y2 = xi * e1 * (1 - e2);
            return xi * xi * xi * e1 * e1;
        case 1: x1 = xi; x2 = xi * e1; y1 = xi * (1 - e1 * e2 * e3); y2 = xi * e1 * e2 * (1 - e3); break;
        case 2: x1 = xi * (1 - e1 * e2); x2 = xi * e1 * (1 - e2); y1 = xi; y2 = xi * e1 * e2 * e3; break;
        case 3: x1 = xi * (1 - e1 * e2 * e3); x2 = xi * e1 * e2 * (1 - e3); y1 = xi; y2 = xi * e1; break;
        default: x1 = xi * (1 - e1 * e2 * e3); x2 = xi * e1 * (1 - e2 * e3); y1 = xi; y2 = xi * e1 * e2; break;
        }
        return xi * xi * xi * e1 * e1 * e2;
    }
    if (reg == 0) {
        x1 = xi; x2 = xi * e1; y1 = xi * e2; y2 = xi * e2 * e3;
    } else {
        x1 = xi * e2; x2 = xi * e2 * e3; y1 = xi; y2 = xi * e1;
    }
    return xi * xi * xi * e2;
}

}  // namespace gca
