/*
 * gca_curved.h -- C-ABI of libgca for curved (quadratic) triangles
 * (Section 6).
 *
 * Triangle t is the image of the reference triangle under the quadratic map
 * Phi_t that interpolates its corners X0, X1, X2 and one point per edge
 * X0-X1, X1-X2, X2-X0 at the edge midpoints.  With the reference point
 * s = (s1, s2), 0 <= s2 <= s1 <= 1, and its barycentric coordinates
 * (l0, l1, l2) = (1 - s1, s1 - s2, s2):
 *     Phi(s) = sum_a l_a (2 l_a - 1) X_a + 4 l0 l1 X3 + 4 l1 l2 X4 + 4 l2 l0 X5,
 * the normal n(s) = dPhi/ds1 x dPhi/ds2 (a quadratic polynomial, evaluated by
 * interpolating its values at the six nodes, Section 6) and the Gramian
 * gamma(s) = |n(s)|.  The basis functions are the mapped nodal functions
 * phi_a o Phi = l_a (Section 6), or their sum, the piecewise-constant
 * function of the triangle.
 *
 * Conventions are those of gca.h: GCA_OK or a negative gca_status, arguments
 * validated before device work is queued, device pointers owned by the
 * caller, work queued on the given stream without synchronisation.
 */
#ifndef GCA_CURVED_H
#define GCA_CURVED_H

#include <stdint.h>

#include "gca.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Galerkin moments of m pairs of curved triangles (Section 6, the double
 * integral over the reference triangles with both Gramians):
 *     M_k[a][b] = int int l_a(x) kappa(Phi_t(x), Phi_s(y)) l_b(y) gamma_t(x) gamma_s(y) dy dx,
 * t = I[k], s = J[k], a and b their corners in mesh order, with
 *     op 0: kappa = g(x, y) = 1 / (4 pi |x - y|)            (single layer),
 *     op 1: kappa = n_s(y) . (x - y) / (4 pi |x - y|^3)      (double layer,
 *           the unit normal n / gamma of t_j's orientation; Section 1).
 * Pairs with a common corner (identical, common edge, common vertex, by the
 * corner ids) take the Sauter-Schwab maps on the reference coordinates with
 * q_s Gauss points in each of the four variables, corners reordered so that
 * the shared ones come first (identical: mesh order; edge: the shared corners
 * by ascending id, then the third; vertex: the shared one, then the cyclic
 * order), the edge points following their edges; the others the regular
 * rule of order q on both triangles (collapsed Gauss q = 1..4, or with
 * sym = 1 the symmetric rules q = 2, 3).  FP64 throughout.
 * nodes: device FP64, nn x 3; tri6: device int32, nt x 6 (X0, X1, X2, then
 *       the points of the edges X0-X1, X1-X2, X2-X0; nodes shared by
 *       neighbouring triangles make the surface closed).
 * I, J: device int32, m triangle ids each; an id outside [0, nt) gives NaN.
 * basis 0: out[k] = sum over a, b of M_k[a][b] (piecewise-constant basis);
 * basis 1: out[9 k + 3 a + b] = M_k[a][b] (mapped nodal basis).
 * out: device FP64, m or 9 m values.
 * Errors: GCA_EINVAL (NULL pointers, m < 0, nt < 1, unsupported op, basis,
 * q, sym or q_s outside 1..32), GCA_EHIP. */
gca_status gca_curved_entries(const double *nodes, const int32_t *tri6, int64_t nt, const int32_t *I,
                              const int32_t *J, int64_t m, int32_t op, int32_t basis, int32_t q, int32_t sym,
                              int32_t q_s, double *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif
